// Panel extraction and Cols(A^(p,q)) selection.
//
// Selection (Table 1; Sec. 3.1 column-based scheme; Sec. 5.1 stage 1) runs
// over the whole panel at once, on a bitmap of the panel's column ids: one
// bit per global id, set for the ids present in the panel.  A prefix sum of
// the per-word popcounts gives every present column its packed position,
// and because column blocks are contiguous id ranges the positions are
// already grouped block by block in ascending id order; block_off[q] is the
// rank of block q's first column id.
//
// The bitmap is built from a copy of the panel's column ids grouped by bins
// of 2^17 ids (made once, at the first selection: a stable radix sort on the
// bin).  A workgroup takes a chunk of one bin, sets the bits of its ids in a
// 16 KB bitmap in LDS (integer OR: the result does not depend on the order)
// and ORs the non-zero words into the global bitmap, so nothing is written
// at random into global memory.  The scan's down pass writes the word table
// used by the remap and clears the bitmap for the next selection.
#include <algorithm>
#include <vector>

#include "plan.hpp"
#include "scan.hpp"

namespace shiro {

namespace {

__global__ void k_rebase(const int64_t* __restrict__ src, int64_t n, int64_t* __restrict__ dst) {
  const int64_t base = src[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i] - base;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Index of the last row r with ptr[r] <= k (ptr non-decreasing, ptr[0] = 0).
__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ ptr, int64_t rows, int64_t k) {
  int64_t lo = 0, hi = rows - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// CSR validation.  bit 1: row_ptr decreasing, bit 2: column out of range,
// bit 4: columns not strictly ascending inside a row.
__global__ void k_check_rows(const int64_t* __restrict__ ptr, int64_t rows, int64_t nnz,
                             int32_t* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < rows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = ptr[i], b = ptr[i + 1];
    if (b < a || a < 0 || b > nnz) atomicOr(flag, 1);
  }
}

__global__ void k_check_cols(const int64_t* __restrict__ ptr, const int32_t* __restrict__ col,
                             int64_t rows, int64_t nnz, int64_t n_cols, int32_t* flag) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = col[k];
    if (c < 0 || (int64_t)c >= n_cols) atomicOr(flag, 2);
    if (k > 0) {
      const int64_t r = row_of(ptr, rows, k);
      if (ptr[r] != k && col[k - 1] >= c) atomicOr(flag, 4);
    }
  }
}

// Per-block nonzero counts: a workgroup-private histogram in LDS, then one
// integer add per bin (integer sums: the result is order independent).
__global__ __launch_bounds__(kBlock) void k_block_nnz(const int32_t* __restrict__ col, int64_t nnz,
                                                      int64_t K, int32_t P,
                                                      unsigned long long* out) {
  extern __shared__ uint32_t hist[];
  for (int i = threadIdx.x; i < P; i += kBlock) hist[i] = 0;
  __syncthreads();
  for (int64_t k = blockIdx.x * (int64_t)kBlock + threadIdx.x; k < nnz; k += (int64_t)gridDim.x * kBlock)
    atomicAdd(&hist[(int64_t)col[k] / K], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += kBlock)
    if (hist[i]) atomicAdd(&out[i], (unsigned long long)hist[i]);
}

__global__ void k_block_nnz_global(const int32_t* __restrict__ col, int64_t nnz, int64_t K,
                                   unsigned long long* out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&out[(int64_t)col[k] / K], 1ull);
}

// Zero a byte range (16 bytes per store; the tail byte by byte).
__global__ void k_zero_bytes(uint8_t* __restrict__ p, int64_t n) {
  const int64_t n16 = n >> 4;
  u32x4 z = {0u, 0u, 0u, 0u};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * blockDim.x)
    reinterpret_cast<u32x4*>(p)[i] = z;
  for (int64_t i = (n16 << 4) + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

constexpr int kBinShift = 17;                          // column ids per bin: 2^17
constexpr int kBinWords = 1 << (kBinShift - 5);        // 4096 bitmap words (16 KB)

// Bin of each column id (the sort key of the bin-major copy).
__global__ void k_bin_keys(const int32_t* __restrict__ col, int64_t nnz, uint32_t* __restrict__ key) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    key[k] = (uint32_t)col[k] >> kBinShift;
}

// off[b] = first entry of bin b in the sorted keys (lower bound), off[nbins] = n.
__global__ void k_bin_off(const uint32_t* __restrict__ skey, int64_t n, int64_t nbins, int64_t* __restrict__ off) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b <= nbins;
       b += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)skey[mid] < b) lo = mid + 1; else hi = mid;
    }
    off[b] = lo;
  }
}

// One chunk (bin, begin, end) of the bin-major ids per workgroup: the bits
// of its ids in an LDS bitmap of the bin, then the non-zero words ORed into
// the panel's bitmap.
__global__ __launch_bounds__(kBlock) void k_mark_bins(const int32_t* __restrict__ bcol,
                                                      const int32_t* __restrict__ items,
                                                      uint32_t* __restrict__ bits, int64_t n_words) {
  __shared__ uint32_t lb[kBinWords];
  for (int i = threadIdx.x; i < kBinWords; i += kBlock) lb[i] = 0;
  __syncthreads();
  const int32_t bin = items[3 * blockIdx.x];
  const int64_t b = items[3 * blockIdx.x + 1], e = items[3 * blockIdx.x + 2];
  // four ids in flight per thread
  for (int64_t k0 = b + threadIdx.x; k0 < e; k0 += 4 * kBlock) {
    uint32_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + u * kBlock;
      c[u] = (uint32_t)bcol[k < e ? k : e - 1];  // a repeated id sets a bit already set
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) atomicOr(&lb[(c[u] >> 5) & (kBinWords - 1)], 1u << (c[u] & 31u));
  }
  __syncthreads();
  const int64_t w0 = (int64_t)bin * kBinWords;
  for (int i = threadIdx.x; i < kBinWords; i += kBlock) {
    const uint32_t v = lb[i];
    if (v != 0u && w0 + i < n_words) atomicOr(&bits[w0 + i], v);
  }
}

struct PopcountIn {
  const uint32_t* bits;
  __device__ int64_t operator()(int64_t w) const { return __popc(bits[w]); }
};

// Down pass of the selection scan: a workgroup owns 256 words (one per
// thread).  Its offset is the sum of the earlier tiles' popcount totals
// (summed here, so no separate pass scans the tile totals; the last tile
// also writes U).  It scans its words' popcounts, writes the word table
// entries (bits, packed position of the word's first set bit) that the
// remap reads, clears the bitmap words it read, and compacts the ids of the
// set bits: each lane writes its word's ids into the tile's slice of an LDS
// buffer, then the workgroup copies the slice to unique_cols with
// consecutive lanes on consecutive ids.
constexpr int kSelItems = 1;

__global__ __launch_bounds__(kBlock) void k_select_down(uint32_t* __restrict__ bits, uint32_t* __restrict__ wtab,
                                                        int64_t n_words, const int64_t* __restrict__ tile_sums,
                                                        int64_t* __restrict__ d_U, int32_t* __restrict__ unique_cols) {
  __shared__ int64_t lds[kWavesPerBlock];
  __shared__ int32_t ids[kBlock * kSelItems * 32];  // at most 32 ids per word
  // this tile's offset: the sum of the earlier tiles' totals
  int64_t before = 0;
  for (int64_t i = threadIdx.x; i < (int64_t)blockIdx.x; i += kBlock) before += tile_sums[i];
  int64_t toff;
  (void)block_exclusive_scan<int64_t>(before, lds, &toff);
  const int64_t w0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kSelItems;
  uint32_t v[kSelItems];
  int64_t cnt = 0;
#pragma unroll
  for (int i = 0; i < kSelItems; ++i) {
    v[i] = w0 + i < n_words ? bits[w0 + i] : 0u;
    cnt += __popc(v[i]);
  }
  int64_t tot;
  int32_t o = (int32_t)block_exclusive_scan<int64_t>(cnt, lds, &tot);
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *d_U = toff + tot;
#pragma unroll
  for (int i = 0; i < kSelItems; ++i) {
    const int64_t w = w0 + i;
    if (w < n_words) {
      const u32x2 t = {v[i], (uint32_t)(toff + o)};
      reinterpret_cast<u32x2*>(wtab)[w] = t;
      if (v[i] != 0u) bits[w] = 0u;
    }
    uint32_t m = v[i];
    while (m != 0u) {
      ids[o++] = (int32_t)((w << 5) + __builtin_ctz(m));
      m &= m - 1u;
    }
  }
  __syncthreads();
  for (int32_t q = threadIdx.x; q < (int32_t)tot; q += kBlock) unique_cols[toff + q] = ids[q];
}

// colmap[k] = packed position of col[k] = offset of its word + set bits
// below it; four nonzeros per thread.  The same threads also write
// block_off[q] = packed position of the first column id of block q (U past
// the end) for q = 0..P.
__global__ void k_remap(const int32_t* __restrict__ col, int64_t nnz,
                        const uint32_t* __restrict__ wtab, int32_t* __restrict__ colmap,
                        int64_t n_cols, int64_t K, int32_t P, const int64_t* __restrict__ d_U,
                        int64_t* __restrict__ block_off) {
  const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const u32x2* tab = reinterpret_cast<const u32x2*>(wtab);
  for (int64_t q = t0; q <= P; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c0 = q * K;
    if (c0 >= n_cols) {
      block_off[q] = *d_U;
    } else {
      const u32x2 e = tab[c0 >> 5];
      block_off[q] = (int64_t)e.y + __popc(e.x & ((1u << ((uint32_t)c0 & 31u)) - 1u));
    }
  }
  const bool vec = ((uintptr_t)col % 16 == 0) && ((uintptr_t)colmap % 16 == 0);
  const int64_t n4 = vec ? (nnz >> 2) : 0;
  auto rank = [&](uint32_t c, const u32x2& e) { return e.y + __popc(e.x & ((1u << (c & 31u)) - 1u)); };
  for (int64_t i = t0; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const u32x4 a = reinterpret_cast<const u32x4*>(col)[i];
    const u32x2 e0 = tab[a.x >> 5], e1 = tab[a.y >> 5], e2 = tab[a.z >> 5], e3 = tab[a.w >> 5];
    const u32x4 o = {rank(a.x, e0), rank(a.y, e1), rank(a.z, e2), rank(a.w, e3)};
    reinterpret_cast<u32x4*>(colmap)[i] = o;
  }
  for (int64_t k = (n4 << 2) + t0; k < nnz; k += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = (uint32_t)col[k];
    const u32x2 e = tab[c >> 5];
    colmap[k] = (int32_t)(e.y + __popc(e.x & ((1u << (c & 31u)) - 1u)));
  }
}

unsigned grid_for(int64_t n, int64_t cap = 65536) {
  int64_t g = ceil_div(n > 0 ? n : 1, kBlock);
  return (unsigned)(g < cap ? g : cap);
}

}  // namespace

int launch_rebase_row_ptr(const int64_t* src, int64_t rows, int64_t* dst, hipStream_t s) {
  k_rebase<<<grid_for(rows + 1), kBlock, 0, s>>>(src, rows + 1, dst);
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

int launch_check_csr(const int64_t* row_ptr, const int32_t* col, int64_t rows, int64_t nnz,
                     int64_t n_cols, int32_t* d_flag, hipStream_t s) {
  if (rows > 0) {
    k_check_rows<<<grid_for(rows), kBlock, 0, s>>>(row_ptr, rows, nnz, d_flag);
    SHIRO_LAUNCH_CHECK();
  }
  if (nnz > 0 && rows > 0) {
    k_check_cols<<<grid_for(nnz), kBlock, 0, s>>>(row_ptr, col, rows, nnz, n_cols, d_flag);
    SHIRO_LAUNCH_CHECK();
  }
  return SHIRO_OK;
}

int launch_block_nnz(const int32_t* col, int64_t nnz, int64_t K, int32_t P, int64_t* out,
                     hipStream_t s) {
  k_fill_i64<<<grid_for(P), kBlock, 0, s>>>(out, P, 0);
  SHIRO_LAUNCH_CHECK();
  if (nnz == 0) return SHIRO_OK;
  auto* o = reinterpret_cast<unsigned long long*>(out);
  if (P <= 16384) {
    k_block_nnz<<<grid_for(nnz, 2048), kBlock, (size_t)P * 4, s>>>(col, nnz, K, P, o);
  } else {
    k_block_nnz_global<<<grid_for(nnz), kBlock, 0, s>>>(col, nnz, K, o);
  }
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

namespace {
struct KeepIn {
  const uint8_t* keep;
  uint8_t v;
  __device__ int64_t operator()(int64_t k) const { return keep[k] == v ? 1 : 0; }
};
struct PosOut {
  int64_t* pos;
  __device__ void operator()(int64_t k, int64_t prefix, int64_t) const { pos[k] = prefix; }
};

// Kept nonzero k of the panel goes to position pos[k] of the subset.
__global__ void k_subset_compact(const int32_t* __restrict__ col, const uint8_t* __restrict__ keep, uint8_t v,
                                 const int64_t* __restrict__ pos, int64_t n, int32_t* __restrict__ col_out,
                                 int32_t* __restrict__ vmap) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x)
    if (keep[k] == v) {
      col_out[pos[k]] = col[k];
      vmap[pos[k]] = (int32_t)k;
    }
}

// Subset row pointers: kept nonzeros before each row start.
__global__ void k_subset_rowptr(const int64_t* __restrict__ row_ptr_src, int64_t rows, int64_t nz0,
                                const int64_t* __restrict__ pos, int64_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= rows;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = pos[row_ptr_src[i] - nz0];
}

__global__ void k_compose(int32_t* __restrict__ perm, const int32_t* __restrict__ vmap, int64_t n) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x)
    perm[j] = vmap[perm[j]];
}
}  // namespace

// pos must hold nnz_panel + 1 entries (pos[nnz_panel] = kept count).
int launch_subset(const int64_t* row_ptr_src, int64_t rows, int64_t nz0, int64_t nnz_panel,
                  const int32_t* col_src, const uint8_t* keep, uint8_t keep_val, int64_t* pos,
                  int32_t* col_out, int32_t* vmap, int64_t* row_ptr_out, void* scan_tmp,
                  hipStream_t s) {
  SHIRO_TRY(scan_generic(KeepIn{keep, keep_val}, nnz_panel, PosOut{pos}, pos + nnz_panel, scan_tmp, s));
  if (nnz_panel > 0) {
    k_subset_compact<<<grid_for(nnz_panel), kBlock, 0, s>>>(col_src, keep, keep_val, pos, nnz_panel, col_out, vmap);
    SHIRO_LAUNCH_CHECK();
  }
  k_subset_rowptr<<<grid_for(rows + 1), kBlock, 0, s>>>(row_ptr_src, rows, nz0, pos, row_ptr_out);
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

int launch_compose(int32_t* perm, const int32_t* vmap, int64_t n, hipStream_t s) {
  if (n <= 0) return SHIRO_OK;
  k_compose<<<grid_for(n), kBlock, 0, s>>>(perm, vmap, n);
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

int launch_zero_bytes(uint8_t* p, int64_t n, hipStream_t s) {
  if (n <= 0) return SHIRO_OK;
  k_zero_bytes<<<grid_for(ceil_div(n, 16), 16384), kBlock, 0, s>>>(p, n);
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

// The bin-major copy of the panel's column ids and its chunk list (setup,
// once per plan): a stable radix sort on the bin, then chunks of at most
// `chunk` ids that never cross a bin.
static int build_bins(shiro_plan plan, hipStream_t s) {
  const int64_t nnz = plan->nnz;
  plan->n_mark_items = 0;
  if (nnz == 0) {
    plan->bins_built = true;
    return SHIRO_OK;
  }
  const int64_t nbins = ceil_div(plan->n_cols, (int64_t)1 << kBinShift);
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  SHIRO_TRY(ensure_scratch(plan, 2 * al(nnz * 4) + al((nbins + 1) * 8) + sort_scratch_bytes(nnz)));
  char* p = reinterpret_cast<char*>(plan->scratch);
  uint32_t* key = reinterpret_cast<uint32_t*>(p);
  uint32_t* skey = reinterpret_cast<uint32_t*>(p + al(nnz * 4));
  int64_t* off = reinterpret_cast<int64_t*>(p + 2 * al(nnz * 4));
  void* tmp = p + 2 * al(nnz * 4) + al((nbins + 1) * 8);
  SHIRO_TRY(dev_alloc_n(&plan->bcol, nnz));
  k_bin_keys<<<grid_for(nnz), kBlock, 0, s>>>(plan->col, nnz, key);
  SHIRO_LAUNCH_CHECK();
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < nbins) ++bits;
  SHIRO_TRY(radix_sort_pairs(key, reinterpret_cast<const uint32_t*>(plan->col), skey,
                             reinterpret_cast<uint32_t*>(plan->bcol), nnz, bits, tmp, s));
  k_bin_off<<<grid_for(nbins + 1), kBlock, 0, s>>>(skey, nnz, nbins, off);
  SHIRO_LAUNCH_CHECK();
  std::vector<int64_t> h((size_t)nbins + 1);
  SHIRO_HIP(hipMemcpyAsync(h.data(), off, (size_t)(nbins + 1) * 8, hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  // about one chunk per compute unit, 2048 to 65536 ids each (each chunk
  // ends with a pass over its bin's 4096 bitmap words, so fewer, larger
  // chunks mark faster: 2^24 R-MAT panel 20 us at four per CU, 15 at two)
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(ceil_div(nnz, (int64_t)plan->num_cus), 2048), 65536);
  std::vector<int32_t> items;
  for (int64_t b = 0; b < nbins; ++b)
    for (int64_t st = h[b]; st < h[b + 1]; st += chunk) {
      items.push_back((int32_t)b);
      items.push_back((int32_t)st);
      items.push_back((int32_t)std::min(st + chunk, h[b + 1]));
    }
  plan->n_mark_items = (int32_t)(items.size() / 3);
  SHIRO_TRY(dev_alloc_n(&plan->mark_items, std::max<int64_t>((int64_t)items.size(), 3)));
  if (!items.empty())
    SHIRO_HIP(hipMemcpy(plan->mark_items, items.data(), items.size() * 4, hipMemcpyHostToDevice));
  plan->bins_built = true;
  return SHIRO_OK;
}

int run_select(shiro_plan plan, hipStream_t s, bool sync) {
  const int64_t nw = plan->n_words;
  const int64_t nnz = plan->nnz;
  if (!plan->bins_built) {
    if (!sync) return set_error(SHIRO_ERR_NOT_READY, "select: the bin-major pattern copy is not built");
    SHIRO_TRY(build_bins(plan, s));
  }
  // scratch: [U (int64)] [scan tile sums]
  SHIRO_TRY(ensure_scratch(plan, 256 + scan_scratch_bytes(nw)));  // (sized for 1 item per thread)
  int64_t* d_U = reinterpret_cast<int64_t*>(plan->scratch);
  void* scan_tmp = reinterpret_cast<char*>(plan->scratch) + 256;

  // the bitmap is all zero here: cleared when the plan was made and by
  // every down pass since
  if (plan->n_mark_items > 0) {
    k_mark_bins<<<plan->n_mark_items, kBlock, 0, s>>>(plan->bcol, plan->mark_items, plan->bits, nw);
    SHIRO_LAUNCH_CHECK();
  }
  // per-tile popcount totals, then the down pass (tile offsets, word table,
  // compaction of the ids)
  const int64_t ntiles = scan_tiles_of(nw, kSelItems);
  int64_t* sums = reinterpret_cast<int64_t*>(scan_tmp);
  k_scan_reduce<kSelItems, PopcountIn><<<dim3((unsigned)ntiles), kBlock, 0, s>>>(PopcountIn{plan->bits}, nw, sums);
  SHIRO_LAUNCH_CHECK();
  k_select_down<<<dim3((unsigned)ntiles), kBlock, 0, s>>>(plan->bits, plan->wtab, nw, sums, d_U, plan->unique_cols);
  SHIRO_LAUNCH_CHECK();
  k_remap<<<grid_for(std::max<int64_t>((nnz + 3) / 4, (int64_t)plan->P + 1)), kBlock, 0, s>>>(
      plan->col, nnz, plan->wtab, plan->colmap, plan->n_cols, plan->K, plan->P, d_U, plan->block_off);
  SHIRO_LAUNCH_CHECK();
  if (!sync) return SHIRO_OK;
  SHIRO_HIP(hipMemcpyAsync(plan->h_pinned, plan->block_off, (size_t)(plan->P + 1) * 8,
                           hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  plan->h_block_off.assign(plan->h_pinned, plan->h_pinned + plan->P + 1);
  plan->U = plan->h_block_off[plan->P];
  plan->selected = true;
  return SHIRO_OK;
}

}  // namespace shiro
