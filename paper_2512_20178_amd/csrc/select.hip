// Panel extraction and Cols(A^(p,q)) selection.
//
// Selection (Table 1; Sec. 3.1 column-based scheme; Sec. 5.1 stage 1) runs
// over the whole panel at once: one flag byte per global column id marks the
// columns present in the panel (plain byte stores of 1: idempotent, no
// atomics, so they stay in each XCD's L2 and merge by byte mask on
// write-back), the flags are folded into one bit per id, a prefix sum of the
// per-word popcounts gives every present column its packed position, and
// because column blocks are contiguous id ranges the positions are already
// grouped block by block in ascending id order.  block_off[q] is the rank of
// block q's first column id.
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

// flag[c] = 1 for every column id c of the panel.  Four ids per thread
// (one 16-byte load when the panel's col array allows it).
__global__ void k_mark(const int32_t* __restrict__ col, int64_t nnz, uint8_t* __restrict__ flag) {
  const int64_t n4 = ((uintptr_t)col % 16 == 0) ? (nnz >> 2) : 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const u32x4 c = reinterpret_cast<const u32x4*>(col)[i];
    flag[c.x] = 1;
    flag[c.y] = 1;
    flag[c.z] = 1;
    flag[c.w] = 1;
  }
  for (int64_t k = (n4 << 2) + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x)
    flag[col[k]] = 1;
}

// Zero the flag bytes (16 bytes per store; the tail byte by byte).
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

// Word table: wtab[2 w] = bits of word w (bit b = flag[32 w + b]; the flag
// array is padded to whole words), wtab[2 w + 1] = packed position of the
// word's first set bit.  Interleaved so that the remap reads one 8-byte entry.
// The flags read are cleared again (only the 16-byte pieces that held a 1),
// so the array is all zero between selections; it is cleared once when the
// plan is made.
__global__ void k_fold_flags(uint8_t* __restrict__ flag, int64_t n_words,
                             uint32_t* __restrict__ wtab) {
  const u32x4 zero = {0u, 0u, 0u, 0u};
  for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < n_words;
       w += (int64_t)gridDim.x * blockDim.x) {
    u32x4* f = reinterpret_cast<u32x4*>(flag + (w << 5));
    const u32x4 a = f[0], b = f[1];
    if ((a.x | a.y | a.z | a.w) != 0u) f[0] = zero;
    if ((b.x | b.y | b.z | b.w) != 0u) f[1] = zero;
    const uint32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      // each byte is 0 or 1: gather bit 0 of the four bytes of v[i]
      const uint32_t x = v[i];
      const uint32_t q = (x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u);
      m |= q << (4 * i);
    }
    wtab[2 * w] = m;
  }
}

struct PopcountIn {
  const uint32_t* wtab;
  __device__ int64_t operator()(int64_t w) const { return __popc(wtab[2 * w]); }
};

// Down pass of the selection scan.  A workgroup owns kSelItems*256 words:
// it scans their popcounts (plus the tile offset from the tile scan), writes
// each word's packed offset into the word table, and then compacts the ids
// of the set bits, so that stores of neighbouring ids are neighbours and no
// lane walks a dense word alone.  A sparse tile (most of them: 7% of the
// bits are set on the 2^24 R-MAT panel) is compacted output by output: lane
// t takes outputs t, t+256, ..., finds the word holding each by binary
// search over the tile's word offsets in LDS and the bit inside it by
// popcount halving.  A dense tile is scanned bit by bit, one id per lane.
constexpr int kSelItems = 4;

// Position of the r-th set bit (r counted from 0) of w; r < popcount(w).
__device__ __forceinline__ uint32_t select_bit(uint32_t w, uint32_t r) {
  uint32_t pos = 0;
#pragma unroll
  for (int h = 16; h >= 1; h >>= 1) {
    const uint32_t c = __popc(w & ((1u << h) - 1u));
    const bool up = r >= c;
    r = up ? r - c : r;
    w = up ? w >> h : w;
    pos += up ? (uint32_t)h : 0u;
  }
  return pos;
}

__global__ __launch_bounds__(kBlock) void k_select_down(uint32_t* __restrict__ wtab, int64_t n_words,
                                                        const int64_t* __restrict__ tile_off,
                                                        int32_t* __restrict__ unique_cols) {
  constexpr int TW = kBlock * kSelItems;  // words per tile
  __shared__ int64_t lds[kWavesPerBlock];
  __shared__ uint32_t sbits[TW];
  __shared__ uint32_t spref[TW];  // offset of each word inside the tile
  const int64_t tile0 = (int64_t)blockIdx.x * TW;
  const int64_t base = tile0 + (int64_t)threadIdx.x * kSelItems;
  const int64_t toff = tile_off[blockIdx.x];
  uint32_t bits[kSelItems];
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kSelItems; ++i) {
    bits[i] = (base + i < n_words) ? wtab[2 * (base + i)] : 0u;
    s += __popc(bits[i]);
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan<int64_t>(s, lds, &tot);
#pragma unroll
  for (int i = 0; i < kSelItems; ++i) {
    if (base + i < n_words) wtab[2 * (base + i) + 1] = (uint32_t)(toff + ex);
    sbits[threadIdx.x * kSelItems + i] = bits[i];
    spref[threadIdx.x * kSelItems + i] = (uint32_t)ex;
    ex += __popc(bits[i]);
  }
  __syncthreads();
  const int32_t count = (int32_t)tot;
  if (count <= TW * 4) {  // sparse: walk the outputs
    for (int32_t o = threadIdx.x; o < count; o += kBlock) {
      int32_t lo = 0, hi = TW - 1;  // last word whose offset is <= o
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((int32_t)spref[mid] <= o) lo = mid; else hi = mid - 1;
      }
      const uint32_t b = select_bit(sbits[lo], (uint32_t)(o - (int32_t)spref[lo]));
      unique_cols[toff + o] = (int32_t)(((tile0 + lo) << 5) + b);
    }
  } else {  // dense: walk the bits
    for (int32_t j = threadIdx.x; j < TW * 32; j += kBlock) {
      const int32_t lw = j >> 5;
      const uint32_t b = (uint32_t)j & 31u;
      const uint32_t wb = sbits[lw];
      if ((wb >> b) & 1u) unique_cols[toff + spref[lw] + __popc(wb & ((1u << b) - 1u))] = (int32_t)((tile0 << 5) + j);
    }
  }
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
  for (int64_t i = t0; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    const u32x4 c = reinterpret_cast<const u32x4*>(col)[i];
    const u32x2 e0 = tab[c.x >> 5], e1 = tab[c.y >> 5], e2 = tab[c.z >> 5], e3 = tab[c.w >> 5];
    u32x4 o;
    o.x = e0.y + __popc(e0.x & ((1u << (c.x & 31u)) - 1u));
    o.y = e1.y + __popc(e1.x & ((1u << (c.y & 31u)) - 1u));
    o.z = e2.y + __popc(e2.x & ((1u << (c.z & 31u)) - 1u));
    o.w = e3.y + __popc(e3.x & ((1u << (c.w & 31u)) - 1u));
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

int run_select(shiro_plan plan, hipStream_t s, bool sync) {
  const int64_t nw = plan->n_words;
  const int64_t nnz = plan->nnz;
  // scratch: [U (int64)] [scan tile sums]
  SHIRO_TRY(ensure_scratch(plan, 256 + scan_scratch_bytes(nw)));  // (sized for 1 item per thread)
  int64_t* d_U = reinterpret_cast<int64_t*>(plan->scratch);
  void* scan_tmp = reinterpret_cast<char*>(plan->scratch) + 256;

  // the flag bytes are all zero here: cleared when the plan was made and
  // by every fold since
  if (nnz > 0) {
    k_mark<<<grid_for((nnz + 3) / 4), kBlock, 0, s>>>(plan->col, nnz, plan->flags);
    SHIRO_LAUNCH_CHECK();
  }
  k_fold_flags<<<grid_for(nw), kBlock, 0, s>>>(plan->flags, nw, plan->wtab);
  SHIRO_LAUNCH_CHECK();
  // reduce-then-scan over the word popcounts; the down pass compacts the ids
  const int64_t ntiles = scan_tiles_of(nw, kSelItems);
  int64_t* sums = reinterpret_cast<int64_t*>(scan_tmp);
  k_scan_reduce<kSelItems, PopcountIn><<<dim3((unsigned)ntiles), kBlock, 0, s>>>(PopcountIn{plan->wtab}, nw, sums);
  SHIRO_LAUNCH_CHECK();
  k_scan_tiles<<<1, kBlock, 0, s>>>(sums, ntiles, d_U);
  SHIRO_LAUNCH_CHECK();
  k_select_down<<<dim3((unsigned)ntiles), kBlock, 0, s>>>(plan->wtab, nw, sums, plan->unique_cols);
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
