// Gather, pack and sparse-times-dense kernels of the per-rank path.
//
// Work decomposition: merge path over (row ends, nonzeros) of a CSR-like
// pattern (ptr[0..R], nnz).  Chunk w covers merge items [w*D, (w+1)*D), so
// every wavefront gets the same amount of work whatever the row lengths are
// (power-law rows of tens of thousands of nonzeros are split over many
// wavefronts, empty rows still cost their store).  A row whose items fall in
// more than one chunk leaves one partial sum per chunk in a carry slot; a
// fix-up pass adds the slots of each such row in chunk order and applies the
// output epilogue once.  No floating-point atomics anywhere, so every output
// is reproducible bit for bit.
//
// Lane layout: a dense row is read 16 bytes per lane by `LANES` lanes (tile
// width LANES*16 bytes: 128 float32 columns for 32 lanes); the 64/LANES lane
// groups of a wavefront take consecutive nonzeros of the same row, UNROLL
// deep, and are reduced with cross-lane shuffles when the row ends.  All row
// bookkeeping is wavefront-uniform and lives in scalar registers.
#include <algorithm>
#include <type_traits>
#include <vector>

#include "plan.hpp"
#include "scan.hpp"

namespace shiro {

namespace {

// ---------------------------------------------------------------------------
// work lists
// ---------------------------------------------------------------------------
__global__ void k_merge_path(const int64_t* __restrict__ ptr, int32_t R, int64_t nnz, int64_t D,
                             int32_t W, int32_t* __restrict__ chunk_row,
                             int32_t* __restrict__ chunk_nz) {
  const int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (w > W) return;
  int64_t d = w * D;
  if (d > (int64_t)R + nnz) d = (int64_t)R + nnz;
  // largest i in [0, R] with ptr[i] + i <= d
  int64_t lo = 0, hi = R;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] + mid <= d) lo = mid; else hi = mid - 1;
  }
  chunk_row[w] = (int32_t)lo;
  chunk_nz[w] = (int32_t)(d - lo);
}

// flag[w] = 1 if chunk w starts a row that a later chunk finishes.
__global__ void k_split_flags(const int64_t* __restrict__ ptr, int32_t R,
                              const int32_t* __restrict__ chunk_row,
                              const int32_t* __restrict__ chunk_nz, int32_t W,
                              int32_t* __restrict__ flag) {
  const int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (w >= W) return;
  const int32_t r = chunk_row[w + 1];
  int32_t f = 0;
  if (r < R) {
    const int64_t rs = ptr[r];
    f = (chunk_nz[w + 1] > rs) && (rs >= chunk_nz[w]);
  }
  flag[w] = f;
}

// split[3 pos[w] ..] = (w, last chunk holding row r, r) for flagged chunks.
__global__ void k_split_emit(const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                             const int32_t* __restrict__ chunk_row, int32_t W,
                             int32_t* __restrict__ split) {
  const int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (w >= W || !flag[w]) return;
  const int32_t r = chunk_row[w + 1];
  // last chunk we with chunk_row[we] <= r, i.e. the first with chunk_row[we + 1] > r
  int64_t lo = w + 1, hi = W - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (chunk_row[mid + 1] > r) hi = mid; else lo = mid + 1;
  }
  const int64_t s = pos[w];
  split[3 * s] = (int32_t)w;
  split[3 * s + 1] = (int32_t)lo;
  split[3 * s + 2] = r;
}

__global__ void k_gather_vals(const int32_t* __restrict__ perm, const float* __restrict__ vals,
                              int64_t nnz, float* __restrict__ out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x)
    out[j] = vals[perm[j]];
}

// One value per thread: with four per thread (16-byte index loads) the
// scattered stores ran slower on the MI355X (55 against 44 us for 4.2M
// values), as did a gather through the inverse permutation.
__global__ void k_scatter_vals(const int32_t* __restrict__ perm, const float* __restrict__ in,
                               int64_t nnz, float* __restrict__ out) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x)
    out[perm[j]] = in[j];
}

// ---------------------------------------------------------------------------
// SpMM: out[r, :] = sum_{k in row r} vals[k] * X[idx[k], :]
// ---------------------------------------------------------------------------
// Host-side bundle of the kernel arguments.  The kernels take them as
// separate __restrict__ parameters: that tells the compiler the pattern
// arrays are never written, so wave-uniform reads of them (row pointers,
// chunk bounds) become scalar loads.
struct SpmmArgs {
  const int64_t* ptr;       // R + 1
  const int32_t* idx;       // nnz: row of X to gather
  const float* vals;        // values in pattern order
  const void* D;            // optional: dense row per pattern row, dotted with each gathered row
  int64_t ldd;
  float* dot_out;           // nnz: the dots, in pattern order (when D is set)
  const void* X;            // gathered dense rows
  int64_t ldx;
  void* out;                // R x N, may be null (transposed: dBpacked optional)
  int64_t ldo;
  void* scat;               // transposed only: dB, rows scat_idx[r] (see scat_mode)
  int64_t lds;
  int32_t scat_mode;        // 1: add the row into dB, 2: overwrite the dB row
  const int32_t* scat_idx;  // R
  const int32_t* chunk_row;  // W + 1
  const int32_t* chunk_nz;   // W + 1
  const int32_t* rid;       // nnz: row of each nonzero (only for patterns without empty rows)
  const int32_t* hot_src;   // windowed walk: rows of X kept in LDS (idx = -(slot + 1) reads slot)
  int32_t n_hot;
  float* carry;             // [W][2][N]
  int32_t W, R, N;
  int32_t chunks_per_wave;
  int32_t xcd_remap;
};

#define SHIRO_SPMM_PARAMS(TIN, TOUT)                                                          \
  const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,                           \
      const float *__restrict__ vals, const TIN *__restrict__ D, int64_t ldd,                 \
      float *__restrict__ dot_out,                                                            \
      const TIN *__restrict__ X, int64_t ldx, TOUT *__restrict__ out, int64_t ldo,           \
      TOUT *__restrict__ scat, int64_t lds, const int32_t *__restrict__ scat_idx,             \
      const int32_t *__restrict__ chunk_row, const int32_t *__restrict__ chunk_nz,            \
      const int32_t *__restrict__ rid, float *__restrict__ carry, int32_t W, int32_t R,         \
      int32_t N, int32_t cpw, int32_t xcd_remap, int32_t scat_mode,                             \
      const int32_t *__restrict__ hot_src, int32_t n_hot

#define SHIRO_SPMM_ARGS(TIN, TOUT, a)                                                          \
  (a).ptr, (a).idx, (a).vals, reinterpret_cast<const TIN*>((a).D), (a).ldd, (a).dot_out,      \
      reinterpret_cast<const TIN*>((a).X), (a).ldx,                                            \
      reinterpret_cast<TOUT*>((a).out), (a).ldo, reinterpret_cast<TOUT*>((a).scat), (a).lds,   \
      (a).scat_idx, (a).chunk_row, (a).chunk_nz, (a).rid, (a).carry, (a).W, (a).R, (a).N,     \
      (a).chunks_per_wave, (a).xcd_remap, (a).scat_mode, (a).hot_src, (a).n_hot

#define SHIRO_SPMM_NAMES                                                                       \
  ptr, idx, vals, D, ldd, dot_out, X, ldx, out, ldo, scat, lds, scat_idx, chunk_row, chunk_nz, rid, \
      carry, W, R, N, cpw, xcd_remap, scat_mode, hot_src, n_hot

template <typename TOUT, int VEC>
__device__ __forceinline__ void epilogue_row(TOUT* __restrict__ out, int64_t ldo, TOUT* __restrict__ scat,
                                             int64_t lds, const int32_t* __restrict__ scat_idx,
                                             int32_t scat_mode, int32_t r, int64_t c,
                                             const float (&acc)[VEC]) {
  if (out) Elem<TOUT>::template store<VEC>(out + (int64_t)r * ldo + c, acc);
  if (scat && scat_mode == 2) {
    Elem<TOUT>::template store<VEC>(scat + (int64_t)scat_idx[r] * lds + c, acc);
  } else if (scat) {
    TOUT* o = scat + (int64_t)scat_idx[r] * lds + c;
    float cur[VEC];
    Elem<TOUT>::template load<VEC>(o, cur);
#pragma unroll
    for (int e = 0; e < VEC; ++e) cur[e] += acc[e];
    Elem<TOUT>::template store<VEC>(o, cur);
  }
}

// Logical workgroup index: with xcd_remap, workgroups that the dispatcher
// places on the same XCD (round robin over 8) get a contiguous index range,
// so each XCD's L2 serves a contiguous range of rows.
__device__ __forceinline__ int32_t logical_block(int32_t remap) {
  const int32_t b = blockIdx.x, g = gridDim.x;
  if (!remap || (g & 7)) return b;
  return (b & 7) * (g >> 3) + (b >> 3);
}

// With DOT (one column tile only), each gathered row is also dotted with the
// pattern row's own dense row D[r]: in the transposed product this is the
// gradient of the values, dvals = dY[row] . Bpacked[u], computed from the
// same dY gathers (no second pass over the nonzeros).
template <typename TIN, typename TOUT, int LANES, int VEC, int UNROLL, bool DOT, int SCAT>
__global__ __launch_bounds__(kBlock) void k_spmm(SHIRO_SPMM_PARAMS(TIN, TOUT)) {
  constexpr int G = kWave / LANES;
  constexpr int STEP = G * UNROLL;
  const int lane = lane_id();
  const int g = lane / LANES;
  const int li = lane % LANES;
  const int64_t c = (int64_t)blockIdx.y * (LANES * VEC) + (int64_t)li * VEC;
  const bool cvalid = c < N;
  const int64_t cl = cvalid ? c : 0;  // idle lanes read an in-bounds column

  const int32_t gw = uniform(logical_block(xcd_remap) * kWavesPerBlock + wave_id());
  const int32_t w_begin = gw * cpw;
  const int32_t w_end = min(w_begin + cpw, W);

  for (int32_t w = w_begin; w < w_end; ++w) {
    const int32_t i0 = chunk_row[w], i1 = chunk_row[w + 1];
    const int64_t j0 = chunk_nz[w], j1 = chunk_nz[w + 1];
    if (i0 >= R) continue;
    int64_t rs = ptr[i0], re = ptr[i0 + 1];
    int32_t sidx = SCAT ? scat_idx[i0] : 0;
    // Indices and values of a row's first step, prefetched during the last
    // step of the previous row (so short rows do not wait for them).
    int32_t xi[UNROLL];
    float v[UNROLL];
    bool ok[UNROLL];
    bool have = false;
    for (int32_t r = i0; r <= i1 && r < R; ++r) {
      if (r == i1 && j1 <= rs) break;  // chunk holds nothing of row i1
      const int64_t kb = rs > j0 ? rs : j0;
      const int64_t ke = re < j1 ? re : j1;
      const bool head = (r == i0) && (j0 > rs);
      const bool tail = (r == i1);
      const bool complete = !head && !tail;
      // the next row of the chunk starts where this one ends
      const bool has_next = (r + 1 <= i1) && (r + 1 < R);
      const int64_t re2 = has_next ? ptr[r + 2] : re;
      const int32_t sidx2 = (SCAT && has_next) ? scat_idx[r + 1] : 0;
      const int64_t ke2 = re2 < j1 ? re2 : j1;
      const bool next_nonempty = has_next && ke2 > re;
      // Load order matters: loads retire in issue order for the wait
      // counter, so the first step's indices are issued before the row's own
      // dense rows (D, the add-scatter target), and nothing reads those until
      // the gathers are in flight — the gathers then wait on the indices only.
      if (!have && kb < ke) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int64_t kk = kb + u * G + g;
          ok[u] = kk < ke;
          const int64_t kc = ok[u] ? kk : ke - 1;
          xi[u] = idx[kc];
          v[u] = vals[kc];
        }
      }
      have = false;
      // the add-scatter target is read now so its latency hides behind the gathers
      float pre[VEC];
      if constexpr (SCAT == 1) {
        if (complete) Elem<TOUT>::template load<VEC>(scat + (int64_t)sidx * lds + cl, pre);
      }
      float acc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
      float d[VEC];  // lanes past N read column 0; their dots are masked below
      if constexpr (DOT) Elem<TIN>::template load<VEC>(D + (int64_t)r * ldd + cl, d);
      // Software pipeline: the index/value loads of the next step (or of the
      // next row's first step) are issued while this step's row gathers are
      // in flight.  All loads are unconditional (idle slots re-read a valid
      // nonzero, a cache hit) so the compiler can count outstanding loads
      // instead of draining them; idle slots are masked by selects.
      for (int64_t k = kb; k < ke; k += STEP) {
        float x[UNROLL][VEC];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          Elem<TIN>::template load<VEC>(X + (int64_t)xi[u] * ldx + cl, x[u]);
        const bool same_row = k + STEP < ke;
        const bool pf = same_row || next_nonempty;
        const int64_t nb = same_row ? k + STEP : (next_nonempty ? re : kb);
        const int64_t nl = same_row ? ke : (next_nonempty ? ke2 : ke);
        int32_t xin[UNROLL];
        float vn[UNROLL];
        bool okn[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int64_t kk = nb + u * G + g;
          okn[u] = pf && kk < nl;
          const int64_t kc = kk < nl ? kk : nl - 1;
          xin[u] = idx[kc];
          vn[u] = vals[kc];
        }
        have = !same_row && next_nonempty;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const float t = fmaf(v[u], x[u][e], acc[e]);
            acc[e] = ok[u] ? t : acc[e];
          }
        if constexpr (DOT) {
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            float q = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e) q = fmaf(d[e], x[u][e], q);
            q = group_sum<LANES>(cvalid ? q : 0.f);
            if (li == LANES - 1 && ok[u]) dot_out[k + u * G + g] = q;
          }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          xi[u] = xin[u];
          v[u] = vn[u];
          ok[u] = okn[u];
        }
      }
      // combine the lane groups (fixed pairing order)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = groups_sum<LANES>(acc[e]);
      if (g == 0 && cvalid) {
        if (complete) {
          if (out) Elem<TOUT>::template store<VEC>(out + (int64_t)r * ldo + c, acc);
          if constexpr (SCAT == 1) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) pre[e] += acc[e];
            Elem<TOUT>::template store<VEC>(scat + (int64_t)sidx * lds + c, pre);
          } else if constexpr (SCAT == 2) {
            Elem<TOUT>::template store<VEC>(scat + (int64_t)sidx * lds + c, acc);
          }
        } else {
          float* cs = carry + ((int64_t)w * 2 + (head ? 0 : 1)) * N + c;
          Elem<float>::template store<VEC>(cs, acc);
        }
      }
      rs = re;
      re = re2;
      sidx = sidx2;
    }
  }
}

// Variant for short rows: lane group g of a wavefront takes rows i0+g,
// i0+g+G, ... of the chunk, UNROLL nonzeros per step, so a wavefront keeps G
// rows in flight instead of one.  Each group reads the row pointers of its
// next row at the start of the current one and that row's first indices
// during the current row's last step, so a short row costs one dependent
// round trip (its gathers).  Row bookkeeping is per group (vector
// registers); groups diverge only in their trip counts.  Sums inside a row
// keep a fixed order, so results stay reproducible.
template <typename TIN, typename TOUT, int LANES, int VEC, int UNROLL, bool DOT, int SCAT>
__global__ __launch_bounds__(kBlock) void k_spmm_grp(SHIRO_SPMM_PARAMS(TIN, TOUT)) {
  constexpr int G = kWave / LANES;
  const int lane = lane_id();
  const int g = lane / LANES;
  const int li = lane % LANES;
  const int64_t c = (int64_t)blockIdx.y * (LANES * VEC) + (int64_t)li * VEC;
  const bool cvalid = c < N;
  const int64_t cl = cvalid ? c : 0;

  const int32_t gw = uniform(logical_block(xcd_remap) * kWavesPerBlock + wave_id());
  const int32_t w_begin = gw * cpw;
  const int32_t w_end = min(w_begin + cpw, W);

  for (int32_t w = w_begin; w < w_end; ++w) {
    const int32_t i0 = chunk_row[w], i1 = chunk_row[w + 1];
    const int64_t j0 = chunk_nz[w], j1 = chunk_nz[w + 1];
    int32_t r = i0 + g;
    if (r > i1 || r >= R) continue;
    int64_t rs = ptr[r], re = ptr[r + 1];
    int32_t xi[UNROLL];
    float v[UNROLL];
    bool ok[UNROLL];
    bool have = false;
    for (; r <= i1 && r < R; r += G) {
      if (r == i1 && j1 <= rs) break;  // chunk holds nothing of row i1
      const int64_t kb = rs > j0 ? rs : j0;
      const int64_t ke = re < j1 ? re : j1;
      const bool head = (r == i0) && (j0 > rs);
      const bool tail = (r == i1);
      const bool complete = !head && !tail;
      const int32_t sidx = SCAT ? scat_idx[r] : 0;
      // indices first, then the group's next row pointers, then the row's
      // own dense rows (loads retire in issue order for the wait counter)
      if (!have && kb < ke) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int64_t kk = kb + u;
          ok[u] = kk < ke;
          const int64_t kc = ok[u] ? kk : ke - 1;
          xi[u] = idx[kc];
          v[u] = vals[kc];
        }
      }
      have = false;
      const int32_t rn = r + G;
      const bool has_next = rn <= i1 && rn < R;
      const int64_t rsn = has_next ? ptr[rn] : re;
      const int64_t ren = has_next ? ptr[rn + 1] : re;
      float pre[VEC];
      if constexpr (SCAT == 1) {
        if (complete) Elem<TOUT>::template load<VEC>(scat + (int64_t)sidx * lds + cl, pre);
      }
      float d[VEC];  // lanes past N read column 0; their dots are masked below
      if constexpr (DOT) Elem<TIN>::template load<VEC>(D + (int64_t)r * ldd + cl, d);
      float acc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
      for (int64_t k = kb; k < ke; k += UNROLL) {
        float x[UNROLL][VEC];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          Elem<TIN>::template load<VEC>(X + (int64_t)xi[u] * ldx + cl, x[u]);
        // next step of this row, or the first step of the group's next row
        const bool same_row = k + UNROLL < ke;
        const int64_t kbn = rsn > j0 ? rsn : j0;
        const int64_t ken = ren < j1 ? ren : j1;
        const bool next_nonempty = has_next && !(rn == i1 && j1 <= rsn) && kbn < ken;
        const bool pf = same_row || next_nonempty;
        const int64_t nb = same_row ? k + UNROLL : (next_nonempty ? kbn : kb);
        const int64_t nl = same_row ? ke : (next_nonempty ? ken : ke);
        int32_t xin[UNROLL];
        float vn[UNROLL];
        bool okn[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int64_t kk = nb + u;
          okn[u] = pf && kk < nl;
          const int64_t kc = kk < nl ? kk : nl - 1;
          xin[u] = idx[kc];
          vn[u] = vals[kc];
        }
        have = !same_row && next_nonempty;
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const float t = fmaf(v[u], x[u][e], acc[e]);
            acc[e] = ok[u] ? t : acc[e];
          }
        if constexpr (DOT) {
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            float q = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e) q = fmaf(d[e], x[u][e], q);
            q = group_sum<LANES>(cvalid ? q : 0.f);
            if (li == LANES - 1 && ok[u]) dot_out[k + u] = q;
          }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          xi[u] = xin[u];
          v[u] = vn[u];
          ok[u] = okn[u];
        }
      }
      if (cvalid) {
        if (complete) {
          if (out) Elem<TOUT>::template store<VEC>(out + (int64_t)r * ldo + c, acc);
          if constexpr (SCAT == 1) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) pre[e] += acc[e];
            Elem<TOUT>::template store<VEC>(scat + (int64_t)sidx * lds + c, pre);
          } else if constexpr (SCAT == 2) {
            Elem<TOUT>::template store<VEC>(scat + (int64_t)sidx * lds + c, acc);
          }
        } else {
          float* cs = carry + ((int64_t)w * 2 + (head ? 0 : 1)) * N + c;
          Elem<float>::template store<VEC>(cs, acc);
        }
      }
      rs = rsn;
      re = ren;
    }
  }
}

// Nonzero walk.  Lane group g of a wavefront owns whole chunks and walks
// their nonzeros UNROLL at a time without regard to row boundaries, so it
// keeps UNROLL dense rows in flight whatever the row lengths (wave-per-row
// and group-per-row kernels stall once per row, and the short rows of
// power-law patterns dominate).  rid[k] is the row of nonzero k; a row's
// sum is written when the walk reaches a nonzero of another row or the
// chunk's end, and rows the walk steps over (no nonzeros) are written as
// zeros.  Rows cut by the chunk's ends go to its carry slots as in k_spmm:
// the first row's piece (empty or not) when that row began in an earlier
// chunk, the last row's piece when the chunk holds any of it.  A group's
// chunks are consecutive, so its nonzeros form one contiguous run and each
// step's indices are loaded one step ahead, across chunk ends too.  Sums
// inside a row keep pattern order, so results stay reproducible.  Rows
// written once (the output, overwritten dB rows) and the dense rows D read
// once are marked non-temporal, so they do not push the gathered rows out
// of the caches (on the 2^24 R-MAT panel this took the transposed product
// without dvals from 469 to 344 us).
template <typename TIN, typename TOUT, int LANES, int VEC, int UNROLL, bool DOT, int SCAT>
__global__ __launch_bounds__(kBlock) void k_spmm_flat(SHIRO_SPMM_PARAMS(TIN, TOUT)) {
  constexpr int G = kWave / LANES;
  const int lane = lane_id();
  const int g = lane / LANES;
  const int li = lane % LANES;
  const int64_t c = (int64_t)blockIdx.y * (LANES * VEC) + (int64_t)li * VEC;
  const bool cvalid = c < N;
  const int64_t cl = cvalid ? c : 0;

  const int64_t worker = (int64_t)uniform(logical_block(xcd_remap) * kWavesPerBlock + wave_id()) * G + g;
  const int64_t wb = worker * cpw;
  const int64_t we = wb + cpw < W ? wb + cpw : W;
  if (wb >= we) return;  // whole lane groups leave; the others use no cross-group lane ops
  const int64_t kend = chunk_nz[we];
  int32_t xi[UNROLL], ri[UNROLL];
  float v[UNROLL];
  if (chunk_nz[wb] < kend) {
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t kk = chunk_nz[wb] + u;
      const int64_t kc = kk < kend ? kk : kend - 1;
      xi[u] = idx[kc];
      ri[u] = rid[kc];
      v[u] = vals[kc];
    }
  }
  for (int64_t w = wb; w < we; ++w) {
    const int32_t i0 = chunk_row[w], i1 = chunk_row[w + 1];
    const int64_t j0 = chunk_nz[w], j1 = chunk_nz[w + 1];
    if (i0 >= R) break;
    const bool has_head = j0 > ptr[i0];
    // rows below row_end whose ends fall in this chunk are complete; `next`
    // is the first of them not written yet
    const int32_t row_end = i1 < R ? i1 : R;
    int32_t next = has_head ? i0 + 1 : i0;
    float* const head_slot = carry + (w * 2) * N + c;
    float* const tail_slot = carry + (w * 2 + 1) * N + c;
    if (has_head && ptr[i0 + 1] <= j0 && cvalid) {  // row i0 holds nothing here
      float z[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) z[e] = 0.f;
      Elem<float>::template store<VEC>(head_slot, z);
    }
    // a complete row's sum: into the output, and into (or onto) its dB row
    auto put = [&](int32_t r, int32_t sidx, const float(&a)[VEC], bool zero) {
      if (out) Elem<TOUT>::template store_nt<VEC>(out + (int64_t)r * ldo + c, a);
      if constexpr (SCAT == 1) {
        if (!zero) {
          float pre[VEC];
          Elem<TOUT>::template load<VEC>(scat + (int64_t)sidx * lds + c, pre);
#pragma unroll
          for (int e = 0; e < VEC; ++e) pre[e] += a[e];
          Elem<TOUT>::template store<VEC>(scat + (int64_t)sidx * lds + c, pre);
        }
      } else if constexpr (SCAT == 2) {
        Elem<TOUT>::template store_nt<VEC>(scat + (int64_t)sidx * lds + c, a);
      }
    };
    // complete rows [next, lim) hold no nonzeros
    auto zero_rows = [&](int32_t lim) {
      for (; next < lim; ++next) {
        if (!cvalid) continue;
        float z[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) z[e] = 0.f;
        put(next, SCAT ? scat_idx[next] : 0, z, true);
      }
    };
    int32_t cur = -1, scur = 0;  // open row and its scatter row
    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
    auto flush = [&]() {
      if (!cvalid) return;
      if (cur == i0 && has_head) Elem<float>::template store<VEC>(head_slot, acc);
      else if (cur == i1) Elem<float>::template store<VEC>(tail_slot, acc);
      else put(cur, scur, acc, false);
    };
    for (int64_t k = j0; k < j1; k += UNROLL) {
      bool ok[UNROLL];
      float x[UNROLL][VEC];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        ok[u] = k + u < j1;
        Elem<TIN>::template load<VEC>(X + (int64_t)xi[u] * ldx + cl, x[u]);
      }
      float d[DOT ? UNROLL : 1][VEC];  // lanes past N read column 0; their dots are masked below
      if constexpr (DOT) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) Elem<TIN>::template load_nt<VEC>(D + (int64_t)ri[u] * ldd + cl, d[u]);
      }
      int32_t sc[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) sc[u] = SCAT ? scat_idx[ri[u]] : 0;
      // the next step: the rest of this chunk, else the next chunk's start
      const int64_t kn = k + UNROLL < j1 ? k + UNROLL : j1;
      int32_t xin[UNROLL], rin[UNROLL];
      float vn[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        const int64_t kk = kn + u;
        const int64_t kc = kk < kend ? kk : kend - 1;
        xin[u] = idx[kc];
        rin[u] = rid[kc];
        vn[u] = vals[kc];
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        if (ok[u] && ri[u] != cur) {
          if (cur >= 0) flush();
          zero_rows(ri[u]);
          cur = ri[u];
          scur = sc[u];
          if (next <= cur) next = cur + 1;
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const float t = fmaf(v[u], x[u][e], acc[e]);
          acc[e] = ok[u] ? t : acc[e];
        }
        if constexpr (DOT) {
          float q = 0.f;
#pragma unroll
          for (int e = 0; e < VEC; ++e) q = fmaf(d[u][e], x[u][e], q);
          q = group_sum<LANES>(cvalid ? q : 0.f);
          if (li == LANES - 1 && ok[u]) dot_out[k + u] = q;
        }
      }
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        xi[u] = xin[u];
        ri[u] = rin[u];
        v[u] = vn[u];
      }
    }
    if (cur >= 0) flush();
    zero_rows(row_end);
  }
}

// Nonzero walk with windowed index streams.  Same walk, carries and output
// order as k_spmm_flat, but a lane group no longer issues one vector load per
// nonzero for each of its index, row-id and value streams: every LANES steps'
// worth of those (a window of LANES consecutive nonzeros) come in with one
// coalesced load per stream, lane li holding nonzero kw + li, and each step
// takes its UNROLL slots from the window by lane permutes (ds_bpermute, the
// LDS crossbar, not the texture path).  On gfx950 a wavefront-wide vector
// load costs the texture addresser about the same whether it fetches 4 or 16
// bytes per lane, and the per-nonzero index loads outnumbered the row
// gathers three to one.  The window after the current one is loaded a whole
// window ahead.  With DOT, the dense row D[r] is loaded only when the row
// changes (runs of a packed column's nonzeros share it), and the dots are
// collected in the window's lanes and written with one store per window.
// With n_hot > 0 the workgroup first copies rows hot_src[0..n_hot) of X (its
// column tile) into LDS, and an index -(slot + 1) in idx reads that slot
// instead of X: the most referenced rows are then served from LDS (the
// tuning knob lds_rows; the index arrays with marked slots are built at
// setup).
template <typename T>
__device__ __forceinline__ T lane_pull(int src_lane, T v) {
  static_assert(sizeof(T) == 4, "32-bit values");
  return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(src_lane << 2, __builtin_bit_cast(int, v)));
}

template <typename TIN, typename TOUT, int LANES, int VEC, int UNROLL, bool DOT, int SCAT>
__device__ __forceinline__ void spmm_win_body(SHIRO_SPMM_PARAMS(TIN, TOUT)) {
  constexpr int G = kWave / LANES;
  constexpr int WIN = LANES;          // nonzeros per window and lane group
  constexpr int WS = WIN / UNROLL;    // steps per window
  static_assert(WIN % UNROLL == 0, "window");
  const int lane = lane_id();
  const int g = lane / LANES;
  const int li = lane % LANES;
  const int base_lane = g * LANES;
  const int32_t c = (int32_t)blockIdx.y * (LANES * VEC) + li * VEC;  // below N
  const bool cvalid = c < N;
  const int32_t cl = cvalid ? c : 0;

  // hot rows: slot h holds the tile's LANES*VEC elements of X row hot_src[h]
  extern __shared__ __align__(16) unsigned char hot_lds[];
  TIN* const hot = reinterpret_cast<TIN*>(hot_lds);
  constexpr int TW = LANES * VEC;
  if (n_hot > 0) {
    const int64_t c0 = (int64_t)blockIdx.y * TW;
    for (int i = threadIdx.x; i < n_hot * LANES; i += kBlock) {
      const int h = i / LANES, l = i % LANES;
      const int64_t cc = c0 + (int64_t)l * VEC;
      TIN* dst = hot + (int64_t)h * TW + l * VEC;
      if (cc < N) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) dst[e] = X[(int64_t)hot_src[h] * ldx + cc + e];
      }
    }
    __syncthreads();
  }
  const int64_t worker = (int64_t)uniform(logical_block(xcd_remap) * kWavesPerBlock + wave_id()) * G + g;
  const int64_t wb = worker * cpw;
  const int64_t we = wb + cpw < W ? wb + cpw : W;
  if (wb >= we) return;  // whole lane groups leave; the others permute inside their own lanes only
  for (int64_t w = wb; w < we; ++w) {
    const int32_t i0 = chunk_row[w], i1 = chunk_row[w + 1];
    const int64_t j0 = chunk_nz[w], j1 = chunk_nz[w + 1];
    if (i0 >= R) break;
    const bool has_head = j0 > ptr[i0];
    const int32_t row_end = i1 < R ? i1 : R;
    int32_t next = has_head ? i0 + 1 : i0;
    // carry slots of this chunk, addressed where used (at its ends only), so
    // that no registers hold them through the walk
    auto head_slot = [&]() { return carry + (w * 2) * N + c; };
    auto tail_slot = [&]() { return carry + (w * 2 + 1) * N + c; };
    if (has_head && ptr[i0 + 1] <= j0 && cvalid) {  // row i0 holds nothing here
      float z[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) z[e] = 0.f;
      Elem<float>::template store<VEC>(head_slot(), z);
    }
    auto put = [&](int32_t r, int32_t sidx, const float(&a)[VEC], bool zero) {
      if (out) Elem<TOUT>::template store_nt<VEC>(out + (int64_t)r * ldo + c, a);
      if constexpr (SCAT == 1) {
        if (!zero) {
          float pre[VEC];
          Elem<TOUT>::template load<VEC>(scat + (int64_t)sidx * lds + c, pre);
#pragma unroll
          for (int e = 0; e < VEC; ++e) pre[e] += a[e];
          Elem<TOUT>::template store<VEC>(scat + (int64_t)sidx * lds + c, pre);
        }
      } else if constexpr (SCAT == 2) {
        Elem<TOUT>::template store_nt<VEC>(scat + (int64_t)sidx * lds + c, a);
      }
    };
    auto zero_rows = [&](int32_t lim) {
      for (; next < lim; ++next) {
        if (!cvalid) continue;
        float z[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) z[e] = 0.f;
        put(next, SCAT ? scat_idx[next] : 0, z, true);
      }
    };
    int32_t cur = -1, scur = 0;
    float acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
    auto flush = [&]() {
      if (!cvalid) return;
      if (cur == i0 && has_head) Elem<float>::template store<VEC>(head_slot(), acc);
      else if (cur == i1) Elem<float>::template store<VEC>(tail_slot(), acc);
      else put(cur, scur, acc, false);
    };
    if (j0 < j1) {
      // window q of the chunk: lane li holds nonzero j0 + q WIN + li (clamped
      // to the chunk's last nonzero; clamped slots are masked below)
      auto wload = [&](int64_t kw, int32_t& wi, int32_t& wr, float& wv, int32_t& wsc) {
        const int64_t kk = kw + li;
        const int64_t kc = kk < j1 ? kk : j1 - 1;
        wi = idx[kc];
        wr = rid[kc];
        wv = vals[kc];
        if constexpr (SCAT != 0) wsc = scat_idx[wr];
      };
      int32_t ci, cr, csc = 0, ni, nr, nsc = 0;
      float cv, nv;
      wload(j0, ci, cr, cv, csc);
      wload(j0 + WIN, ni, nr, nv, nsc);
      // slots of the first step
      int32_t xi[UNROLL], ri[UNROLL], sc[UNROLL];
      float v[UNROLL];
#pragma unroll
      for (int u = 0; u < UNROLL; ++u) {
        xi[u] = lane_pull(base_lane + u, ci);
        ri[u] = lane_pull(base_lane + u, cr);
        v[u] = lane_pull(base_lane + u, cv);
        sc[u] = SCAT ? lane_pull(base_lane + u, csc) : 0;
      }
      float dl[DOT ? VEC : 1];  // D row of the previous slot and its row
      int32_t dr = -1;
      float mydot = 0.f;        // this lane's nonzero of the window: its dot
      int s = 0;                // step inside the window
      for (int64_t k = j0; k < j1; k += UNROLL) {
        bool ok[UNROLL];
        float x[UNROLL][VEC];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          ok[u] = k + u < j1;
          if (xi[u] < 0) Elem<TIN>::template load<VEC>(hot + (int64_t)(-xi[u] - 1) * TW + li * VEC, x[u]);
          else Elem<TIN>::template load<VEC>(X + (int64_t)xi[u] * ldx + cl, x[u]);
        }
        float d[DOT ? UNROLL : 1][VEC];
        if constexpr (DOT) {
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            const int32_t rp = u == 0 ? dr : ri[u - 1];
            if (ri[u] != rp) {
              Elem<TIN>::template load_nt<VEC>(D + (int64_t)ri[u] * ldd + cl, d[u]);
            } else {
#pragma unroll
              for (int e = 0; e < VEC; ++e) d[u][e] = u == 0 ? dl[e] : d[u - 1][e];
            }
          }
#pragma unroll
          for (int e = 0; e < VEC; ++e) dl[e] = d[UNROLL - 1][e];
          dr = ri[UNROLL - 1];
        }
        // the next step's slots: the current window, or the next one when
        // this step ends the window (then the windows move up by one)
        const int sn = s + 1 == WS ? 0 : s + 1;
        if (sn == 0) {
          ci = ni; cr = nr; cv = nv; csc = nsc;
          wload(k + UNROLL + WIN, ni, nr, nv, nsc);
        }
        int32_t xin[UNROLL], rin[UNROLL], scn[UNROLL];
        float vn[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int src = base_lane + sn * UNROLL + u;
          xin[u] = lane_pull(src, ci);
          rin[u] = lane_pull(src, cr);
          vn[u] = lane_pull(src, cv);
          scn[u] = SCAT ? lane_pull(src, csc) : 0;
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          if (ok[u] && ri[u] != cur) {
            if (cur >= 0) flush();
            zero_rows(ri[u]);
            cur = ri[u];
            scur = sc[u];
            if (next <= cur) next = cur + 1;
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
          }
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const float t = fmaf(v[u], x[u][e], acc[e]);
            acc[e] = ok[u] ? t : acc[e];
          }
          if constexpr (DOT) {
            float q = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e) q = fmaf(d[u][e], x[u][e], q);
            q = group_sum<LANES>(cvalid ? q : 0.f);
            q = lane_pull(base_lane + LANES - 1, q);
            mydot = li == s * UNROLL + u ? q : mydot;
          }
        }
        if constexpr (DOT) {
          // the window's dots, one store per window
          if (sn == 0 || k + UNROLL >= j1) {
            const int64_t kd = k - (int64_t)s * UNROLL + li;
            if (kd < j1 && kd <= k + UNROLL - 1) dot_out[kd] = mydot;
          }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          xi[u] = xin[u];
          ri[u] = rin[u];
          v[u] = vn[u];
          sc[u] = scn[u];
        }
        s = sn;
      }
    }
    if (cur >= 0) flush();
    zero_rows(row_end);
  }
}

template <typename TIN, typename TOUT, int LANES, int VEC, int UNROLL, bool DOT, int SCAT>
__global__ __launch_bounds__(kBlock) void k_spmm_win(SHIRO_SPMM_PARAMS(TIN, TOUT)) {
  spmm_win_body<TIN, TOUT, LANES, VEC, UNROLL, DOT, SCAT>(SHIRO_SPMM_NAMES);
}

// The same walk compiled for eight wavefronts per SIMD (at most 64 VGPRs; a
// few values spill).  The fused transposed product in FP32 with one nonzero
// per step and lane groups of 16 or more has short rows (a few nonzeros per
// packed column), so its waves spend most of their time waiting on loads and
// more of them in flight pay: on the 2^24 R-MAT panel 516 -> 503 us at
// N = 128 and 331 -> 326 us at N = 64, results bit-identical.  With 8-lane
// groups (N = 32) the spills cost more than the extra waves gain (243 -> 248
// us), and the forward walks lose to the spills too, so they keep the
// default budget.
template <typename TIN, typename TOUT, int LANES, int VEC, int UNROLL, bool DOT, int SCAT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_spmm_win_w8(
    SHIRO_SPMM_PARAMS(TIN, TOUT)) {
  spmm_win_body<TIN, TOUT, LANES, VEC, UNROLL, DOT, SCAT>(SHIRO_SPMM_NAMES);
}

// Rows cut by chunk boundaries.  split[3 i] = first chunk ws, split[3 i + 1]
// = last chunk we, split[3 i + 2] = row r.  The row's pieces are the tail
// slot of ws and the head slots of ws+1 .. we, summed in that order.  The
// list holds the splits of at most kFixupSmall pieces first (nearly all of
// them): the first blocks give each of those to one lane group (32 or 64
// lanes), which adds the pieces one after another.  Each of the remaining
// (hub rows cut by many chunks) gets a whole workgroup: slice s sums pieces
// s, s + S, s + 2S, ... in order, then slice 0 adds the S slice sums in
// order.  The path depends only on the piece count, so every result is
// reproducible.  The epilogue is applied once.
template <typename TIN, typename TOUT, int VEC>
__global__ __launch_bounds__(kBlock) void k_fixup(SHIRO_SPMM_PARAMS(TIN, TOUT),
                                                  const int32_t* __restrict__ split, int32_t nsplit,
                                                  int32_t nsmall) {
  __shared__ float part[kBlock * VEC];
  const int32_t t = threadIdx.x;
  // lane groups: 32 lanes when a row fits in 32*VEC columns, else 64
  const int32_t L = (N <= 32 * VEC) ? 32 : 64;
  const int32_t per_block = kBlock / L;
  const int32_t small_blocks = (nsmall + per_block - 1) / per_block;
  if ((int32_t)blockIdx.x < small_blocks) {
    const int64_t i = (int64_t)blockIdx.x * per_block + t / L;
    const int32_t gl = t % L;
    if (i >= nsmall) return;
    const int32_t ws = split[3 * i], we = split[3 * i + 1], r = split[3 * i + 2];
    const int32_t np = we - ws + 1;
    for (int64_t c = (int64_t)gl * VEC; c < N; c += (int64_t)L * VEC) {
      float p[kFixupSmall][VEC];
#pragma unroll
      for (int q = 0; q < kFixupSmall; ++q) {
        if (q < np) {
          const int64_t slot = q == 0 ? (int64_t)ws * 2 + 1 : (int64_t)(ws + q) * 2;
          Elem<float>::template load<VEC>(carry + slot * N + c, p[q]);
        }
      }
      float acc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = p[0][e];
#pragma unroll
      for (int q = 1; q < kFixupSmall; ++q) {
        if (q < np) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e] += p[q][e];
        }
      }
      epilogue_row<TOUT, VEC>(out, ldo, scat, lds, scat_idx, scat_mode, r, c, acc);
    }
    return;
  }
  // one workgroup per long split
  const int32_t lanes_per_row = (int32_t)min((int64_t)kBlock, ((int64_t)N + VEC - 1) / VEC);
  const int32_t S = kBlock / lanes_per_row;
  const int32_t sl = t / lanes_per_row, li = t % lanes_per_row;
  for (int64_t i = nsmall + (int64_t)blockIdx.x - small_blocks; i < nsplit;
       i += (int64_t)gridDim.x - small_blocks) {
    const int32_t ws = split[3 * i], we = split[3 * i + 1], r = split[3 * i + 2];
    const int32_t np = we - ws + 1;
    for (int64_t c0 = 0; c0 < N; c0 += (int64_t)lanes_per_row * VEC) {
      const int64_t c = c0 + (int64_t)li * VEC;
      float acc[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
      if (sl < S && c < N) {
        for (int32_t q = sl; q < np; q += S) {
          const int64_t slot = q == 0 ? (int64_t)ws * 2 + 1 : (int64_t)(ws + q) * 2;
          float p[VEC];
          Elem<float>::template load<VEC>(carry + slot * N + c, p);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e] += p[e];
        }
      }
      __syncthreads();
#pragma unroll
      for (int e = 0; e < VEC; ++e) part[t * VEC + e] = acc[e];
      __syncthreads();
      if (sl == 0 && c < N) {
        for (int32_t q = 1; q < S; ++q)
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e] += part[(q * lanes_per_row + li) * VEC + e];
        epilogue_row<TOUT, VEC>(out, ldo, scat, lds, scat_idx, scat_mode, r, c, acc);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// SDDMM: dvals[k] = dY[row(k), :] . Bp[colmap[k], :]
// ---------------------------------------------------------------------------
struct SddmmArgs {
  const int64_t* ptr;
  const int32_t* idx;
  const void* dY;
  int64_t lddy;
  const void* Bp;
  int64_t ldp;
  float* dvals;
  const int32_t* out_map;  // optional: dvals index of each pattern nonzero (subset plans)
  const int32_t* chunk_row;
  const int32_t* chunk_nz;
  int32_t W, R, N;
  int32_t chunks_per_wave;
  int32_t xcd_remap;
};

template <typename TIN, int LANES, int VEC, int UNROLL>
__global__ __launch_bounds__(kBlock) void k_sddmm(
    const int64_t* __restrict__ ptr, const int32_t* __restrict__ idx, const TIN* __restrict__ dY,
    int64_t lddy, const TIN* __restrict__ Bp, int64_t ldp, float* __restrict__ dvals,
    const int32_t* __restrict__ out_map, const int32_t* __restrict__ chunk_row,
    const int32_t* __restrict__ chunk_nz, int32_t W, int32_t R, int32_t N, int32_t cpw, int32_t xcd_remap) {
  constexpr int G = kWave / LANES;
  constexpr int TW = LANES * VEC;
  constexpr int STEP = G * UNROLL;
  const int lane = lane_id();
  const int g = lane / LANES;
  const int li = lane % LANES;
  const int ntiles = (N + TW - 1) / TW;
  const int64_t c0 = (int64_t)li * VEC;

  const int32_t gw = uniform(logical_block(xcd_remap) * kWavesPerBlock + wave_id());
  const int32_t w_begin = gw * cpw;
  const int32_t w_end = min(w_begin + cpw, W);

  for (int32_t w = w_begin; w < w_end; ++w) {
    const int32_t i0 = chunk_row[w], i1 = chunk_row[w + 1];
    const int64_t j0 = chunk_nz[w], j1 = chunk_nz[w + 1];
    int64_t rs = i0 < R ? ptr[i0] : 0;
    for (int32_t r = i0; r <= i1 && r < R; ++r) {
      const int64_t re = ptr[r + 1];
      const int64_t kb = rs > j0 ? rs : j0;
      const int64_t ke = re < j1 ? re : j1;
      rs = re;
      if (kb >= ke) continue;
      // first column tile of dY row r stays in registers for the whole row
      float y0[VEC];
      Elem<TIN>::template load<VEC>(dY + (int64_t)r * lddy + (c0 < N ? c0 : 0), y0);
      if (c0 >= N) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) y0[e] = 0.f;
      }
      for (int64_t k = kb; k < ke; k += STEP) {
        int32_t xi[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          const int64_t kk = k + u * G + g;
          xi[u] = idx[kk < ke ? kk : ke - 1];
        }
        float part[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          float b[VEC];
          Elem<TIN>::template load<VEC>(Bp + (int64_t)xi[u] * ldp + (c0 < N ? c0 : 0), b);
          part[u] = 0.f;
#pragma unroll
          for (int e = 0; e < VEC; ++e) part[u] = fmaf(y0[e], b[e], part[u]);
        }
        for (int t = 1; t < ntiles; ++t) {
          const int64_t ct = (int64_t)t * TW + c0;
          const bool cv = ct < N;
          float y[VEC];
          Elem<TIN>::template load<VEC>(dY + (int64_t)r * lddy + (cv ? ct : 0), y);
#pragma unroll
          for (int u = 0; u < UNROLL; ++u) {
            float b[VEC];
            Elem<TIN>::template load<VEC>(Bp + (int64_t)xi[u] * ldp + (cv ? ct : 0), b);
            float q = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e) q = fmaf(y[e], b[e], q);
            part[u] += cv ? q : 0.f;
          }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
          part[u] = group_sum<LANES>(part[u]);
          const int64_t kk = k + u * G + g;
          if (li == LANES - 1 && kk < ke) dvals[out_map ? (int64_t)out_map[kk] : kk] = part[u];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// pack: Bp[u, :] = B[uc[u], :]  (bit-exact row gather)
// ---------------------------------------------------------------------------
template <typename T, int LANES, int VEC, int UNROLL>
__global__ __launch_bounds__(kBlock) void k_pack(const int32_t* __restrict__ uc, int64_t U,
                                                 const T* __restrict__ B, int64_t ldb,
                                                 T* __restrict__ Bp, int64_t ldp, int32_t N) {
  constexpr int G = kWave / LANES;
  constexpr int TW = LANES * VEC;
  const int lane = lane_id();
  const int g = lane / LANES;
  const int li = lane % LANES;
  const int64_t groups = (int64_t)gridDim.x * kWavesPerBlock * G;
  const int64_t gid = ((int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6)) * G + g;
  for (int64_t u0 = gid; u0 < U; u0 += groups * UNROLL) {
    int32_t src[UNROLL];
#pragma unroll
    for (int q = 0; q < UNROLL; ++q) {
      const int64_t u = u0 + q * groups;
      src[q] = u < U ? uc[u] : -1;
    }
    for (int64_t c = (int64_t)li * VEC; c < N; c += TW) {
#pragma unroll
      for (int q = 0; q < UNROLL; ++q) {
        const int64_t u = u0 + q * groups;
        if (src[q] >= 0) RawVec<T, VEC>::copy(B + (int64_t)src[q] * ldb + c, Bp + u * ldp + c);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// one launch per column block (the baseline of the batched form)
// ---------------------------------------------------------------------------
// Block q's own CSR over its (row, block) entries, in the block-major order of
// the row-based structures: x in [off[q] + q, off[q+1] + q] is entry
// i = x - off[q] - q of block q, and its row pointer is rebased to the
// block's first nonzero.
__global__ void k_pb_ptr(const int64_t* __restrict__ rb_ptr, const int64_t* __restrict__ off, int32_t P,
                         int64_t total, int64_t* __restrict__ pb_ptr) {
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total;
       x += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = P - 1;  // last q with off[q] + q <= x
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (off[mid] + mid <= x) lo = mid; else hi = mid - 1;
    }
    const int64_t e0 = off[lo];
    pb_ptr[x] = rb_ptr[e0 + (x - e0 - lo)] - rb_ptr[e0];
  }
}

// For block-major nonzero t: its packed row (colmap of its CSR position) and
// its entry counted from the block's first entry.
__global__ void k_pb_fill(const int32_t* __restrict__ rb_rid, const int32_t* __restrict__ rb_perm,
                          const int32_t* __restrict__ colmap, const int64_t* __restrict__ off, int32_t P,
                          int64_t nnz, int32_t* __restrict__ pb_idx, int32_t* __restrict__ pb_rid) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = rb_rid[t];
    int32_t lo = 0, hi = P - 1;  // last q with off[q] <= j
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (off[mid] <= j) lo = mid; else hi = mid - 1;
    }
    pb_idx[t] = colmap[rb_perm[t]];
    pb_rid[t] = (int32_t)(j - off[lo]);
  }
}

template <typename T>
__global__ void k_zero_rows(T* __restrict__ Y, int64_t rows, int64_t ldy, int32_t N) {
  const int64_t total = rows * (int64_t)N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / N, c = i - r * N;
    Y[r * ldy + c] = T(0);
  }
}

__global__ void k_round_rows(const float* __restrict__ src, int64_t lds, bf16_t* __restrict__ dst,
                             int64_t ldd, int64_t rows, int32_t N) {
  const int64_t total = rows * (int64_t)N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / N, c = i - r * N;
    dst[r * ldd + c] = f32_to_bf16(src[r * lds + c]);
  }
}

// ---------------------------------------------------------------------------
// setup kernels: transposed pattern and per-block segments
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ ptr, int64_t rows, int64_t k) {
  int64_t lo = 0, hi = rows - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (ptr[mid] <= k) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_iota(uint32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (uint32_t)i;
}

// After sorting (colmap, k): row of each entry and the first entry of each
// packed column (every packed column has at least one entry).
__global__ void k_transpose_finish(const uint32_t* __restrict__ skeys,
                                   const uint32_t* __restrict__ perm, int64_t nnz,
                                   const int64_t* __restrict__ row_ptr, int64_t rows, int64_t U,
                                   int32_t* __restrict__ trow, int64_t* __restrict__ tptr) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * blockDim.x) {
    trow[j] = (int32_t)row_of(row_ptr, rows, perm[j]);
    if (j == 0 || skeys[j] != skeys[j - 1]) tptr[skeys[j]] = j;
    if (j == nnz - 1) tptr[U] = nnz;
  }
}

// rid[k] = the row holding entry k of a CSR pattern (binary search).
__global__ void k_row_ids(const int64_t* __restrict__ ptr, int64_t rows, int64_t n, int32_t* __restrict__ rid) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    rid[k] = (int32_t)row_of(ptr, rows, k);
}

// Segment starts: first nonzero of a row, or a change of column block.
__global__ void k_seg_flags(const int64_t* __restrict__ row_ptr, int64_t rows,
                            const int32_t* __restrict__ col, int64_t nnz, int64_t K,
                            int32_t* __restrict__ flag) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    int32_t f = 1;
    if (k > 0) {
      const int64_t r = row_of(row_ptr, rows, k);
      f = (row_ptr[r] == k) || ((int64_t)col[k] / K != (int64_t)col[k - 1] / K);
    }
    flag[k] = f;
  }
}

__global__ void k_seg_emit(const int32_t* __restrict__ flag, const int64_t* __restrict__ pos,
                           int64_t nnz, const int64_t* __restrict__ row_ptr, int64_t rows,
                           const int32_t* __restrict__ col, int64_t K, uint32_t* __restrict__ key,
                           int32_t* __restrict__ sbeg, int32_t* __restrict__ srow) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nnz;
       k += (int64_t)gridDim.x * blockDim.x) {
    if (!flag[k]) continue;
    const int64_t s = pos[k];
    sbeg[s] = (int32_t)k;
    srow[s] = (int32_t)row_of(row_ptr, rows, k);
    key[s] = (uint32_t)((int64_t)col[k] / K);
  }
}

__global__ void k_seg_gather(const uint32_t* __restrict__ order, int64_t nseg,
                             const int32_t* __restrict__ sbeg, const int32_t* __restrict__ srow,
                             int64_t nnz, int32_t* __restrict__ obeg, int32_t* __restrict__ oend,
                             int32_t* __restrict__ orow) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < nseg;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t s = order[j];
    obeg[j] = sbeg[s];
    oend[j] = (s + 1 < nseg) ? sbeg[s + 1] : (int32_t)nnz;
    orow[j] = srow[s];
  }
}

// off[q] = first sorted segment of block q (lower bound), off[P] = nseg.
__global__ void k_seg_off(const uint32_t* __restrict__ skey, int64_t nseg, int32_t P,
                          int64_t* __restrict__ off) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q > P) return;
  int64_t lo = 0, hi = nseg;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)skey[mid] < q) lo = mid + 1; else hi = mid;
  }
  off[q] = lo;
}

__global__ void k_fill_random_f32(float* p, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    p[i] = (float)((int64_t)(z >> 40) - (1ll << 23)) * (1.0f / 8388608.0f);
  }
}

unsigned grid_for(int64_t n, int64_t cap = 65536) {
  int64_t g = ceil_div(n > 0 ? n : 1, kBlock);
  return (unsigned)(g < cap ? g : cap);
}

// ---------------------------------------------------------------------------
// row-based scheme: setup of the block-major copy and of the sum pattern
// ---------------------------------------------------------------------------
// For nonzero t of the block-major order: its entry j (ptr[j] <= t <
// ptr[j+1]), its CSR position and its global column id.
__global__ void k_rb_fill(const int64_t* __restrict__ ptr, int64_t R, const int32_t* __restrict__ seg_begin,
                          const int32_t* __restrict__ col, int64_t nnz, int32_t* __restrict__ perm,
                          int32_t* __restrict__ col_bm, int32_t* __restrict__ rid) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz;
       t += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = R - 1;  // last j with ptr[j] <= t
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (ptr[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const int32_t k = seg_begin[lo] + (int32_t)(t - ptr[lo]);
    perm[t] = k;
    col_bm[t] = col[k];
    rid[t] = (int32_t)lo;
  }
}

// agg_idx[c] = block-major position of CSR-order segment c; row_csr[c] = its row.
__global__ void k_rb_agg(const int32_t* __restrict__ seg_csr, const int32_t* __restrict__ seg_row,
                         int64_t R, int32_t* __restrict__ agg_idx, int32_t* __restrict__ row_csr,
                         float* __restrict__ ones) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < R;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = seg_csr[j];
    agg_idx[c] = (int32_t)j;
    row_csr[c] = seg_row[j];
    ones[j] = 1.0f;
  }
}

// agg_ptr[i] = first CSR-order segment of row i (row_csr is non-decreasing).
__global__ void k_rb_agg_ptr(const int32_t* __restrict__ row_csr, int64_t R, int64_t rows,
                             int64_t* __restrict__ agg_ptr) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= rows;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = R;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)row_csr[mid] < i) lo = mid + 1; else hi = mid;
    }
    agg_ptr[i] = lo;
  }
}

struct SegLen {
  const int32_t* b;
  const int32_t* e;
  __device__ int64_t operator()(int64_t j) const { return (int64_t)e[j] - b[j]; }
};
struct OutPtr {
  int64_t* p;
  __device__ void operator()(int64_t j, int64_t prefix, int64_t) const { p[j] = prefix; }
};

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------
template <typename T>
bool aligned16(const void* p, int64_t ld) {
  return ((uintptr_t)p % 16 == 0) && ((ld * (int64_t)sizeof(T)) % 16 == 0);
}

// Vector width in elements: 16 bytes when N, ld and base allow it, else 1.
template <typename T>
int vec_for(int32_t N, std::initializer_list<std::pair<const void*, int64_t>> mats) {
  constexpr int V = Elem<T>::kVec16;
  if (N % V) return 1;
  for (auto& m : mats)
    if (m.first && !aligned16<T>(m.first, m.second)) return 1;
  return V;
}

// Persistent grid over `workers_per_block` workers per workgroup (its
// wavefronts, or their lane groups): at most wg_per_cu workgroups per CU,
// each worker owning *chunks_per_worker consecutive chunks.
int grid_waves(shiro_plan plan, const shiro_tuning_t& t, int32_t W, int32_t workers_per_block,
               int32_t* chunks_per_worker, unsigned* blocks) {
  const int64_t max_blocks = (int64_t)plan->num_cus * (t.wg_per_cu > 0 ? t.wg_per_cu : 8);
  int64_t nb = ceil_div(W, workers_per_block);
  if (nb > max_blocks) nb = max_blocks;
  if (nb < 1) nb = 1;
  *chunks_per_worker = (int32_t)ceil_div(W, nb * workers_per_block);
  nb = ceil_div(ceil_div(W, *chunks_per_worker), workers_per_block);
  if (t.xcd_remap) nb = ceil_div(nb, 8) * 8;  // whole rounds of the 8 XCDs
  *blocks = (unsigned)nb;
  return SHIRO_OK;
}

template <typename TIN, typename TOUT, int VEC, bool DOT, int SCAT>
int spmm_dispatch(const shiro_tuning_t& t, dim3 grid, hipStream_t s, const SpmmArgs& a) {
#define SHIRO_SPMM_CASE(L, U)                                                                          \
  if (t.lanes == L && t.unroll == U) {                                                                 \
    if (t.group_rows == 3 && a.rid) {                                                                  \
      const size_t lds_bytes = (size_t)a.n_hot * L * VEC * sizeof(TIN);                               \
      if constexpr (DOT && U == 1 && L >= 16 && std::is_same<TIN, float>::value)                      \
        k_spmm_win_w8<TIN, TOUT, L, VEC, U, DOT, SCAT><<<grid, kBlock, lds_bytes, s>>>(                \
            SHIRO_SPMM_ARGS(TIN, TOUT, a));                                                           \
      else                                                                                             \
        k_spmm_win<TIN, TOUT, L, VEC, U, DOT, SCAT><<<grid, kBlock, lds_bytes, s>>>(                   \
            SHIRO_SPMM_ARGS(TIN, TOUT, a));                                                           \
    } else if (t.group_rows == 2 && a.rid)                                                               \
      k_spmm_flat<TIN, TOUT, L, VEC, U, DOT, SCAT><<<grid, kBlock, 0, s>>>(SHIRO_SPMM_ARGS(TIN, TOUT, a)); \
    else if (t.group_rows)                                                                             \
      k_spmm_grp<TIN, TOUT, L, VEC, U, DOT, SCAT><<<grid, kBlock, 0, s>>>(SHIRO_SPMM_ARGS(TIN, TOUT, a)); \
    else                                                                                               \
      k_spmm<TIN, TOUT, L, VEC, U, DOT, SCAT><<<grid, kBlock, 0, s>>>(SHIRO_SPMM_ARGS(TIN, TOUT, a));     \
    SHIRO_LAUNCH_CHECK();                                                                              \
    return SHIRO_OK;                                                                                   \
  }
  SHIRO_SPMM_CASE(8, 1) SHIRO_SPMM_CASE(8, 2) SHIRO_SPMM_CASE(8, 4)
  SHIRO_SPMM_CASE(16, 1) SHIRO_SPMM_CASE(16, 2) SHIRO_SPMM_CASE(16, 4)
  SHIRO_SPMM_CASE(32, 1) SHIRO_SPMM_CASE(32, 2) SHIRO_SPMM_CASE(32, 4)
  SHIRO_SPMM_CASE(64, 1) SHIRO_SPMM_CASE(64, 2) SHIRO_SPMM_CASE(64, 4)
#undef SHIRO_SPMM_CASE
  return set_error(SHIRO_ERR_UNSUPPORTED, "spmm: no kernel for lanes/unroll");
}

template <typename TIN, int VEC>
int sddmm_dispatch(const shiro_tuning_t& t, dim3 grid, hipStream_t s, const SddmmArgs& a) {
#define SHIRO_SDDMM_CASE(L, U)                                                              \
  if (t.lanes == L && t.unroll == U) {                                                      \
    k_sddmm<TIN, L, VEC, U><<<grid, kBlock, 0, s>>>(                                        \
        a.ptr, a.idx, reinterpret_cast<const TIN*>(a.dY), a.lddy,                           \
        reinterpret_cast<const TIN*>(a.Bp), a.ldp, a.dvals, a.out_map, a.chunk_row,         \
        a.chunk_nz, a.W, a.R, a.N, a.chunks_per_wave, a.xcd_remap);                         \
    SHIRO_LAUNCH_CHECK();                                                                   \
    return SHIRO_OK;                                                                        \
  }
  SHIRO_SDDMM_CASE(8, 1) SHIRO_SDDMM_CASE(8, 2) SHIRO_SDDMM_CASE(8, 4)
  SHIRO_SDDMM_CASE(16, 1) SHIRO_SDDMM_CASE(16, 2) SHIRO_SDDMM_CASE(16, 4)
  SHIRO_SDDMM_CASE(32, 1) SHIRO_SDDMM_CASE(32, 2) SHIRO_SDDMM_CASE(32, 4)
  SHIRO_SDDMM_CASE(64, 1) SHIRO_SDDMM_CASE(64, 2) SHIRO_SDDMM_CASE(64, 4)
#undef SHIRO_SDDMM_CASE
  return set_error(SHIRO_ERR_UNSUPPORTED, "sddmm: no kernel for lanes/unroll");
}

// Lanes actually used: never more than one column tile needs.
int effective_lanes(int lanes, int32_t N, int vec) {
  int need = (int)ceil_div(N, vec);
  int l = lanes;
  while (l > 8 && l / 2 >= need) l /= 2;
  return l;
}

template <typename TIN, typename TOUT>
int run_spmm_family(shiro_plan plan, shiro_tuning_t t, const WorkList* wl, SpmmArgs a, int vec,
                    hipStream_t s) {
  t.lanes = effective_lanes(t.lanes, a.N, vec);
  unsigned nb;
  // the nonzero walk gives each lane group its own chunks
  const int32_t workers = (t.group_rows >= 2 && a.rid) ? kWavesPerBlock * (kWave / t.lanes) : kWavesPerBlock;
  SHIRO_TRY(grid_waves(plan, t, wl->W, workers, &a.chunks_per_wave, &nb));
  const int ntiles = (int)ceil_div(a.N, (int64_t)t.lanes * vec);
  a.xcd_remap = t.xcd_remap;
  if (a.n_hot > 0 && (int64_t)a.n_hot * t.lanes * vec * (int64_t)sizeof(TIN) > 65536)
    return set_error(SHIRO_ERR_UNSUPPORTED, "spmm: lds_rows rows of this width exceed 64 KB of LDS");
  dim3 grid(nb, ntiles);
  constexpr int V16 = Elem<TIN>::kVec16;
  const bool store = a.scat_mode == 2;
  if (a.dot_out) {
    if (ntiles != 1) return set_error(SHIRO_ERR_UNSUPPORTED, "fused dvals needs one column tile");
    if (a.scat && store) {
      if (vec == V16) SHIRO_TRY((spmm_dispatch<TIN, TOUT, V16, true, 2>(t, grid, s, a)));
      else SHIRO_TRY((spmm_dispatch<TIN, TOUT, 1, true, 2>(t, grid, s, a)));
    } else if (a.scat) {
      if (vec == V16) SHIRO_TRY((spmm_dispatch<TIN, TOUT, V16, true, 1>(t, grid, s, a)));
      else SHIRO_TRY((spmm_dispatch<TIN, TOUT, 1, true, 1>(t, grid, s, a)));
    } else {
      if (vec == V16) SHIRO_TRY((spmm_dispatch<TIN, TOUT, V16, true, 0>(t, grid, s, a)));
      else SHIRO_TRY((spmm_dispatch<TIN, TOUT, 1, true, 0>(t, grid, s, a)));
    }
  } else if (a.scat && store) {
    if (vec == V16) SHIRO_TRY((spmm_dispatch<TIN, TOUT, V16, false, 2>(t, grid, s, a)));
    else SHIRO_TRY((spmm_dispatch<TIN, TOUT, 1, false, 2>(t, grid, s, a)));
  } else if (a.scat) {
    if (vec == V16) SHIRO_TRY((spmm_dispatch<TIN, TOUT, V16, false, 1>(t, grid, s, a)));
    else SHIRO_TRY((spmm_dispatch<TIN, TOUT, 1, false, 1>(t, grid, s, a)));
  } else {
    if (vec == V16) SHIRO_TRY((spmm_dispatch<TIN, TOUT, V16, false, 0>(t, grid, s, a)));
    else SHIRO_TRY((spmm_dispatch<TIN, TOUT, 1, false, 0>(t, grid, s, a)));
  }
  if (wl->nsplit == 0) return SHIRO_OK;
  const int fvec = (vec == V16 && (a.N % 4) == 0) ? 4 : 1;
  const int64_t per_block = kBlock / ((a.N <= 32 * fvec) ? 32 : 64);
  const int64_t nbig = (int64_t)wl->nsplit - wl->nsmall;
  const unsigned fb = (unsigned)(ceil_div(wl->nsmall, per_block) + std::min<int64_t>(nbig, 16384));
  if (fvec == 4) {
    k_fixup<TIN, TOUT, 4><<<fb, kBlock, 0, s>>>(SHIRO_SPMM_ARGS(TIN, TOUT, a), wl->split, wl->nsplit, wl->nsmall);
  } else {
    k_fixup<TIN, TOUT, 1><<<fb, kBlock, 0, s>>>(SHIRO_SPMM_ARGS(TIN, TOUT, a), wl->split, wl->nsplit, wl->nsmall);
  }
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

}  // namespace

// ===========================================================================
// host entry points
// ===========================================================================
int build_worklist(const int64_t* ptr, int64_t R, int64_t nnz, int32_t chunk, WorkList* wl,
                   hipStream_t s) {
  wl->chunk = chunk;
  wl->W = (int32_t)ceil_div(R + nnz, chunk);
  SHIRO_TRY(dev_alloc_n(&wl->chunk_row, (int64_t)wl->W + 1));
  SHIRO_TRY(dev_alloc_n(&wl->chunk_nz, (int64_t)wl->W + 1));
  k_merge_path<<<grid_for((int64_t)wl->W + 1, 1 << 20), kBlock, 0, s>>>(
      ptr, (int32_t)R, nnz, chunk, wl->W, wl->chunk_row, wl->chunk_nz);
  SHIRO_LAUNCH_CHECK();
  wl->nsplit = 0;
  if (wl->W == 0) return SHIRO_OK;
  // list of rows cut by chunk boundaries (temporary buffers, freed here)
  int32_t* flag = nullptr;
  int64_t* pos = nullptr;
  void* tmp = nullptr;
  int64_t* h_n = nullptr;
  auto cleanup = [&] {
    dev_free(flag);
    dev_free(pos);
    dev_free(tmp);
    if (h_n) (void)hipHostFree(h_n);
  };
  int rc;
  if ((rc = dev_alloc_n(&flag, wl->W)) || (rc = dev_alloc_n(&pos, (int64_t)wl->W + 1)) ||
      (rc = dev_alloc(&tmp, scan_scratch_bytes(wl->W)))) {
    cleanup();
    return rc;
  }
  if (hipHostMalloc((void**)&h_n, 8, hipHostMallocDefault) != hipSuccess) {
    cleanup();
    return set_error(SHIRO_ERR_OOM, "work list: pinned allocation failed");
  }
  k_split_flags<<<grid_for(wl->W, 1 << 20), kBlock, 0, s>>>(ptr, (int32_t)R, wl->chunk_row,
                                                            wl->chunk_nz, wl->W, flag);
  if ((rc = exclusive_scan_i32_to_i64(flag, wl->W, pos, pos + wl->W, tmp, s)) ||
      hipMemcpyAsync(h_n, pos + wl->W, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return rc ? rc : set_error(SHIRO_ERR_HIP, "work list: split count failed");
  }
  wl->nsplit = (int32_t)*h_n;
  if (wl->nsplit > 0) {
    if ((rc = dev_alloc_n(&wl->split, 3 * (int64_t)wl->nsplit))) {
      cleanup();
      return rc;
    }
    k_split_emit<<<grid_for(wl->W, 1 << 20), kBlock, 0, s>>>(flag, pos, wl->chunk_row, wl->W, wl->split);
  }
  hipError_t e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) return set_error(SHIRO_ERR_HIP, "work list: split list failed");
  wl->nsmall = 0;
  if (wl->nsplit == 0) return SHIRO_OK;
  // order the list: splits of at most kFixupSmall pieces first (setup only)
  std::vector<int32_t> h((size_t)wl->nsplit * 3), o;
  o.reserve(h.size());
  if (hipMemcpy(h.data(), wl->split, h.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(SHIRO_ERR_HIP, "work list: reading the split list failed");
  for (int pass = 0; pass < 2; ++pass)
    for (size_t i = 0; i < (size_t)wl->nsplit; ++i) {
      const bool small = h[3 * i + 1] - h[3 * i] + 1 <= kFixupSmall;
      if (small == (pass == 0)) o.insert(o.end(), h.begin() + 3 * i, h.begin() + 3 * i + 3);
    }
  for (size_t i = 0; i < (size_t)wl->nsplit; ++i)
    if (h[3 * i + 1] - h[3 * i] + 1 <= kFixupSmall) ++wl->nsmall;
  if (hipMemcpy(wl->split, o.data(), o.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return set_error(SHIRO_ERR_HIP, "work list: writing the split list failed");
  return SHIRO_OK;
}

int build_transposed(shiro_plan plan, hipStream_t s) {
  Transposed& tr = plan->tr;
  if (tr.built) return SHIRO_OK;
  const int64_t nnz = plan->nnz, U = plan->U;
  SHIRO_TRY(dev_alloc_n(&tr.ptr, U + 1));
  SHIRO_TRY(dev_alloc_n(&tr.row, nnz > 0 ? nnz : 1));
  SHIRO_TRY(dev_alloc_n(&tr.perm, nnz > 0 ? nnz : 1));
  SHIRO_TRY(dev_alloc_n(&tr.rid, nnz > 0 ? nnz : 1));
  if (nnz == 0) {
    scan_generic(
        [] __device__(int64_t) -> int64_t { return 0; }, 0,
        [] __device__(int64_t, int64_t, int64_t) {}, tr.ptr, nullptr, s);
    tr.built = true;
    return SHIRO_OK;
  }
  // scratch: iota values + sort scratch; the sorted keys are the entries' rows
  const int64_t need = (nnz * 4 + 256) + sort_scratch_bytes(nnz);
  SHIRO_TRY(ensure_scratch(plan, need));
  char* p = reinterpret_cast<char*>(plan->scratch);
  uint32_t* iota = reinterpret_cast<uint32_t*>(p);
  void* sort_tmp = p + (nnz * 4 + 256) / 256 * 256;
  uint32_t* skeys = reinterpret_cast<uint32_t*>(tr.rid);
  k_iota<<<grid_for(nnz), kBlock, 0, s>>>(iota, nnz);
  SHIRO_LAUNCH_CHECK();
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < U) ++bits;
  SHIRO_TRY(radix_sort_pairs(reinterpret_cast<const uint32_t*>(plan->colmap), iota, skeys,
                             reinterpret_cast<uint32_t*>(tr.perm), nnz, bits, sort_tmp, s));
  k_transpose_finish<<<grid_for(nnz), kBlock, 0, s>>>(skeys, reinterpret_cast<uint32_t*>(tr.perm),
                                                       nnz, plan->row_ptr, plan->rows, U, tr.row,
                                                       tr.ptr);
  SHIRO_LAUNCH_CHECK();
  // subset plans read the caller's values through the value map
  if (plan->vmap) SHIRO_TRY(launch_compose(tr.perm, plan->vmap, nnz, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  tr.built = true;
  return SHIRO_OK;
}

int build_segments(shiro_plan plan, hipStream_t s) {
  BlockSegments& sg = plan->seg;
  if (sg.built) return SHIRO_OK;
  const int64_t nnz = plan->nnz;
  const int32_t P = plan->P;
  sg.h_off.assign((size_t)P + 1, 0);
  if (nnz == 0) {
    sg.nseg = 0;
    sg.built = true;
    return SHIRO_OK;
  }
  auto al = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t need = al(nnz * 4) + al(nnz * 8) + al(8) + 3 * al(nnz * 4) + al(nnz * 4) +
                       al(nnz * 4) + al((int64_t)(P + 1) * 8) +
                       std::max(scan_scratch_bytes(nnz), sort_scratch_bytes(nnz));
  SHIRO_TRY(ensure_scratch(plan, need));
  char* p = reinterpret_cast<char*>(plan->scratch);
  auto take = [&](int64_t b) {
    char* r = p;
    p += al(b);
    return r;
  };
  int32_t* flag = reinterpret_cast<int32_t*>(take(nnz * 4));
  int64_t* pos = reinterpret_cast<int64_t*>(take(nnz * 8));
  int64_t* d_n = reinterpret_cast<int64_t*>(take(8));
  uint32_t* key = reinterpret_cast<uint32_t*>(take(nnz * 4));
  int32_t* sbeg = reinterpret_cast<int32_t*>(take(nnz * 4));
  int32_t* srow = reinterpret_cast<int32_t*>(take(nnz * 4));
  uint32_t* iota = reinterpret_cast<uint32_t*>(take(nnz * 4));
  uint32_t* skey = reinterpret_cast<uint32_t*>(take(nnz * 4));
  int64_t* off = reinterpret_cast<int64_t*>(take((int64_t)(P + 1) * 8));
  void* tmp = p;

  k_seg_flags<<<grid_for(nnz), kBlock, 0, s>>>(plan->row_ptr, plan->rows, plan->col, nnz, plan->K,
                                                flag);
  SHIRO_LAUNCH_CHECK();
  SHIRO_TRY(exclusive_scan_i32_to_i64(flag, nnz, pos, d_n, tmp, s));
  SHIRO_HIP(hipMemcpyAsync(plan->h_pinned, d_n, 8, hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  const int64_t nseg = plan->h_pinned[0];
  sg.nseg = nseg;
  k_seg_emit<<<grid_for(nnz), kBlock, 0, s>>>(flag, pos, nnz, plan->row_ptr, plan->rows,
                                               plan->col, plan->K, key, sbeg, srow);
  SHIRO_LAUNCH_CHECK();
  k_iota<<<grid_for(nseg), kBlock, 0, s>>>(iota, nseg);
  SHIRO_LAUNCH_CHECK();
  int bits = 0;
  while (bits < 32 && ((int64_t)1 << bits) < P) ++bits;
  uint32_t* order = reinterpret_cast<uint32_t*>(flag);  // flags no longer needed
  SHIRO_TRY(radix_sort_pairs(key, iota, skey, order, nseg, bits, tmp, s));
  SHIRO_TRY(dev_alloc_n(&sg.seg_row, nseg));
  SHIRO_TRY(dev_alloc_n(&sg.seg_begin, nseg));
  SHIRO_TRY(dev_alloc_n(&sg.seg_end, nseg));
  k_seg_gather<<<grid_for(nseg), kBlock, 0, s>>>(order, nseg, sbeg, srow, nnz, sg.seg_begin,
                                                  sg.seg_end, sg.seg_row);
  SHIRO_LAUNCH_CHECK();
  SHIRO_TRY(dev_alloc_n(&sg.seg_csr, nseg));
  SHIRO_HIP(hipMemcpyAsync(sg.seg_csr, order, (size_t)nseg * 4, hipMemcpyDeviceToDevice, s));
  k_seg_off<<<grid_for((int64_t)P + 1), kBlock, 0, s>>>(skey, nseg, P, off);
  SHIRO_LAUNCH_CHECK();
  std::vector<int64_t> h((size_t)P + 1);
  SHIRO_HIP(hipMemcpyAsync(h.data(), off, (size_t)(P + 1) * 8, hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  sg.h_off = h;
  sg.built = true;
  return SHIRO_OK;
}

int launch_pack(shiro_plan plan, const void* B, int64_t ldb, int32_t N, shiro_dtype dt, void* Bp,
                int64_t ldp, hipStream_t s) {
  const int64_t U = plan->U;
  if (U == 0 || N == 0) return SHIRO_OK;
  // Four workgroups per CU: on the 2^24 R-MAT panel (FP32, N = 128) 2, 4, 8
  // and 16 gave 315, 246, 261 and 270 us -- fewer random rows of the large B
  // in flight at once run faster, down to the point where latency shows.
  // Eight rows per lane group per round: 2, 4 and 8 gave 255, 246 and 242 us
  // (BF16 134, 129 and 124 us; the ER panel 764, 722 and 722 us).
  const unsigned nb = grid_for(U * 8, (int64_t)plan->num_cus * 4);
  if (dt == SHIRO_F32) {
    const int v = vec_for<float>(N, {{B, ldb}, {Bp, ldp}});
    const int64_t lanes = effective_lanes(64, N, v);
    auto go = [&](auto L, auto V) {
      k_pack<float, decltype(L)::value, decltype(V)::value, 8><<<nb, kBlock, 0, s>>>(
          plan->unique_cols, U, (const float*)B, ldb, (float*)Bp, ldp, N);
    };
    if (v == 4) {
      if (lanes <= 8) go(std::integral_constant<int, 8>{}, std::integral_constant<int, 4>{});
      else if (lanes <= 16) go(std::integral_constant<int, 16>{}, std::integral_constant<int, 4>{});
      else if (lanes <= 32) go(std::integral_constant<int, 32>{}, std::integral_constant<int, 4>{});
      else go(std::integral_constant<int, 64>{}, std::integral_constant<int, 4>{});
    } else {
      go(std::integral_constant<int, 64>{}, std::integral_constant<int, 1>{});
    }
  } else {
    const int v = vec_for<bf16_t>(N, {{B, ldb}, {Bp, ldp}});
    const int64_t lanes = effective_lanes(64, N, v);
    auto go = [&](auto L, auto V) {
      k_pack<bf16_t, decltype(L)::value, decltype(V)::value, 8><<<nb, kBlock, 0, s>>>(
          plan->unique_cols, U, (const bf16_t*)B, ldb, (bf16_t*)Bp, ldp, N);
    };
    if (v == 8) {
      if (lanes <= 8) go(std::integral_constant<int, 8>{}, std::integral_constant<int, 8>{});
      else if (lanes <= 16) go(std::integral_constant<int, 16>{}, std::integral_constant<int, 8>{});
      else if (lanes <= 32) go(std::integral_constant<int, 32>{}, std::integral_constant<int, 8>{});
      else go(std::integral_constant<int, 64>{}, std::integral_constant<int, 8>{});
    } else {
      go(std::integral_constant<int, 64>{}, std::integral_constant<int, 1>{});
    }
  }
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

namespace {
// out[r] = sum vals[k] X[idx[k]] over a CSR-like pattern (ptr: R + 1) with
// its work list, for the supported dtype pairs.
int launch_pattern(shiro_plan plan, const shiro_tuning_t& t, const WorkList* wl, const int64_t* ptr,
                   const int32_t* idx, const float* vals, int64_t R, const void* X, int64_t ldx,
                   int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                   hipStream_t s, const int32_t* add_rows = nullptr, const int32_t* rid = nullptr,
                   float* carry = nullptr, const HotRows* hot = nullptr) {
  SpmmArgs a{};
  if (hot) {  // the windowed walk reads the hot rows from LDS
    idx = hot->walk_idx;
    a.hot_src = hot->hot_src;
    a.n_hot = hot->H;
  }
  a.ptr = ptr;
  a.rid = rid;
  a.idx = idx;
  a.vals = vals;
  a.X = X;
  a.ldx = ldx;
  if (add_rows) {  // Y[add_rows[r]] += the sum of row r
    a.scat = Y;
    a.lds = ldy;
    a.scat_idx = add_rows;
    a.scat_mode = 1;
  } else {
    a.out = Y;
    a.ldo = ldy;
  }
  a.chunk_row = wl->chunk_row;
  a.chunk_nz = wl->chunk_nz;
  a.carry = carry ? carry : plan->carry;
  a.W = wl->W;
  a.R = (int32_t)R;
  a.N = N;
  if (in_dt == SHIRO_F32 && out_dt == SHIRO_F32) {
    const int v = vec_for<float>(N, {{X, ldx}, {Y, ldy}});
    return run_spmm_family<float, float>(plan, t, wl, a, v, s);
  }
  if (in_dt == SHIRO_BF16 && out_dt == SHIRO_F32) {
    const int v = vec_for<bf16_t>(N, {{X, ldx}}) == 8 && aligned16<float>(Y, ldy) ? 8 : 1;
    return run_spmm_family<bf16_t, float>(plan, t, wl, a, v, s);
  }
  if (in_dt == SHIRO_BF16 && out_dt == SHIRO_BF16) {
    const int v = vec_for<bf16_t>(N, {{X, ldx}, {Y, ldy}});
    return run_spmm_family<bf16_t, bf16_t>(plan, t, wl, a, v, s);
  }
  return set_error(SHIRO_ERR_UNSUPPORTED, "dtype pair not supported (F32->F32, BF16->F32, BF16->BF16)");
}
}  // namespace

// The plan's values in its own nonzero order: the caller's array at the
// panel's offset, or (subset plans) gathered through the value map.
static const float* plan_values(shiro_plan plan, const float* vals, hipStream_t s) {
  const float* v = vals + plan->nz_begin;
  if (!plan->vmap || plan->nnz == 0) return v;
  k_gather_vals<<<grid_for(plan->nnz), kBlock, 0, s>>>(plan->vmap, v, plan->nnz, plan->svals);
  return plan->svals;
}

int ensure_hot(shiro_plan plan, int kernel, int32_t H, bool allocate, hipStream_t s, const HotRows** out) {
  const auto key = std::make_pair((int32_t)kernel, H);
  auto it = plan->hot.find(key);
  if (it != plan->hot.end()) {
    *out = &it->second;
    return SHIRO_OK;
  }
  if (!allocate) return set_error(SHIRO_ERR_CAPTURING, "spmm: LDS rows of the tuning not prepared before capture");
  if (kernel == SHIRO_KERNEL_SPMM_T && !plan->tr.built) SHIRO_TRY(build_transposed(plan, s));
  const int64_t nnz = plan->nnz;
  const int32_t* src = kernel == SHIRO_KERNEL_SPMM ? plan->colmap : plan->tr.row;
  const int64_t nx = kernel == SHIRO_KERNEL_SPMM ? plan->U : plan->rows;
  std::vector<int32_t> h((size_t)std::max<int64_t>(nnz, 1));
  if (nnz > 0) SHIRO_HIP(hipMemcpyAsync(h.data(), src, (size_t)nnz * 4, hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  // the H most referenced rows (count descending, index ascending)
  std::vector<int64_t> cnt((size_t)std::max<int64_t>(nx, 1), 0);
  for (int64_t k = 0; k < nnz; ++k) ++cnt[(size_t)h[k]];
  std::vector<int32_t> order((size_t)nx);
  for (int64_t x = 0; x < nx; ++x) order[(size_t)x] = (int32_t)x;
  const int64_t take = std::min<int64_t>(H, nx);
  std::partial_sort(order.begin(), order.begin() + take, order.end(), [&](int32_t a, int32_t b) {
    return cnt[(size_t)a] != cnt[(size_t)b] ? cnt[(size_t)a] > cnt[(size_t)b] : a < b;
  });
  int32_t n_hot = 0;
  while (n_hot < take && cnt[(size_t)order[(size_t)n_hot]] > 1) ++n_hot;  // a row read once gains nothing
  std::vector<int32_t> slot((size_t)std::max<int64_t>(nx, 1), -1);
  for (int32_t q = 0; q < n_hot; ++q) slot[(size_t)order[(size_t)q]] = q;
  for (int64_t k = 0; k < nnz; ++k)
    if (slot[(size_t)h[k]] >= 0) h[k] = -(slot[(size_t)h[k]] + 1);
  HotRows hr;
  hr.H = n_hot;
  // nothing is kept unless every step succeeds
  auto fail = [&](int rc) {
    dev_free(hr.walk_idx);
    dev_free(hr.hot_src);
    return rc;
  };
  int rc = dev_alloc_n(&hr.walk_idx, std::max<int64_t>(nnz, 1));
  if (rc == SHIRO_OK) rc = dev_alloc_n(&hr.hot_src, std::max<int32_t>(n_hot, 1));
  if (rc != SHIRO_OK) return fail(rc);
  hipError_t e = hipSuccess;
  if (nnz > 0) e = hipMemcpyAsync(hr.walk_idx, h.data(), (size_t)nnz * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && n_hot > 0)
    e = hipMemcpyAsync(hr.hot_src, order.data(), (size_t)n_hot * 4, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess)
    return fail(set_error(e == hipErrorOutOfMemory ? SHIRO_ERR_OOM : SHIRO_ERR_HIP,
                          std::string("LDS rows: ") + hipGetErrorString(e)));
  *out = &(plan->hot[key] = hr);
  return SHIRO_OK;
}

int ensure_row_rid(shiro_plan plan, bool allocate, hipStream_t s) {
  if (plan->row_rid) return SHIRO_OK;
  if (!allocate) return set_error(SHIRO_ERR_CAPTURING, "spmm: row ids for the nonzero walk not prepared before capture");
  SHIRO_TRY(dev_alloc_n(&plan->row_rid, std::max<int64_t>(plan->nnz, 1)));
  if (plan->nnz > 0) {
    k_row_ids<<<grid_for(plan->nnz), kBlock, 0, s>>>(plan->row_ptr, plan->rows, plan->nnz, plan->row_rid);
    SHIRO_LAUNCH_CHECK();
  }
  return SHIRO_OK;
}

int launch_spmm(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* X,
                int64_t ldx, int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy,
                shiro_dtype out_dt, hipStream_t s) {
  if (plan->rows == 0 || N == 0) return SHIRO_OK;
  const WorkList* wl;
  SHIRO_TRY(ensure_rows_work(plan, t.chunk, !stream_capturing(s), s, &wl));
  if (t.group_rows >= 2) SHIRO_TRY(ensure_row_rid(plan, !stream_capturing(s), s));
  SHIRO_TRY(ensure_carry(plan, (int64_t)wl->W * 2 * N, !stream_capturing(s)));
  const HotRows* hot = nullptr;
  if (t.group_rows == 3 && t.lds_rows > 0)
    SHIRO_TRY(ensure_hot(plan, SHIRO_KERNEL_SPMM, t.lds_rows, !stream_capturing(s), s, &hot));
  const float* v = plan_values(plan, vals, s);
  SHIRO_LAUNCH_CHECK();
  return launch_pattern(plan, t, wl, plan->row_ptr, plan->colmap, v, plan->rows, X, ldx, N, in_dt, Y, ldy,
                        out_dt, s, nullptr, t.group_rows >= 2 ? plan->row_rid : nullptr, nullptr, hot);
}

int launch_spmm_fixed(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* X,
                      int64_t ldx, int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                      float* carry, int64_t carry_cap, hipStream_t s) {
  if (plan->rows == 0 || N == 0) return SHIRO_OK;
  auto it = plan->rows_work.find(t.chunk);
  if (it == plan->rows_work.end() || (t.group_rows >= 2 && !plan->row_rid))
    return set_error(SHIRO_ERR_NOT_READY,
                     "spmm_noalloc: work list of the tuning not built; run shiro_prepare for (N, dtype) first");
  const WorkList* wl = &it->second;
  const int64_t need = (int64_t)wl->W * 2 * N;
  if (need > carry_cap)
    return set_error(SHIRO_ERR_WORKSPACE,
                     "spmm_noalloc: the carry slots need " + std::to_string(need * 4) +
                         " bytes, more than the fixed work area of " + std::to_string(carry_cap * 4) + " bytes");
  const HotRows* hot = nullptr;
  if (t.group_rows == 3 && t.lds_rows > 0) {
    auto ht = plan->hot.find(std::make_pair((int32_t)SHIRO_KERNEL_SPMM, t.lds_rows));
    if (ht == plan->hot.end())
      return set_error(SHIRO_ERR_NOT_READY, "spmm_noalloc: LDS rows of the tuning not built; run shiro_prepare first");
    hot = &ht->second;
  }
  const float* v = plan_values(plan, vals, s);
  SHIRO_LAUNCH_CHECK();
  return launch_pattern(plan, t, wl, plan->row_ptr, plan->colmap, v, plan->rows, X, ldx, N, in_dt, Y, ldy,
                        out_dt, s, nullptr, t.group_rows >= 2 ? plan->row_rid : nullptr, carry, hot);
}

int build_rowbased(shiro_plan plan, hipStream_t s) {
  RowBased& rb = plan->rb;
  if (rb.built) return SHIRO_OK;
  SHIRO_TRY(build_segments(plan, s));
  const BlockSegments& sg = plan->seg;
  const int64_t R = sg.nseg, nnz = plan->nnz, rows = plan->rows;
  const int32_t P = plan->P;
  rb.R = R;
  SHIRO_TRY(dev_alloc_n(&rb.ptr, R + 1));
  SHIRO_TRY(dev_alloc_n(&rb.col, std::max<int64_t>(nnz, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.perm, std::max<int64_t>(nnz, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.rid, std::max<int64_t>(nnz, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.agg_ptr, rows + 1));
  SHIRO_TRY(dev_alloc_n(&rb.agg_rid, std::max<int64_t>(R, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.agg_idx, std::max<int64_t>(R, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.ones, std::max<int64_t>(R, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.vals, std::max<int64_t>(nnz, 1)));
  SHIRO_TRY(dev_alloc_n(&rb.block_off, (int64_t)P + 1));
  SHIRO_TRY(dev_alloc_n(&rb.iota, std::max<int64_t>(rows, 1)));
  if (rows > 0) {
    k_iota<<<grid_for(rows), kBlock, 0, s>>>(reinterpret_cast<uint32_t*>(rb.iota), rows);
    SHIRO_LAUNCH_CHECK();
  }
  SHIRO_HIP(hipMemcpyAsync(rb.block_off, sg.h_off.data(), (size_t)(P + 1) * 8, hipMemcpyHostToDevice, s));
  // the block-major copy: entry j covers nonzeros [ptr[j], ptr[j+1])
  SHIRO_TRY(ensure_scratch(plan, scan_scratch_bytes(std::max<int64_t>(R, 1)) + (std::max<int64_t>(R, 1) * 4 + 256)));
  char* scr = reinterpret_cast<char*>(plan->scratch);
  int32_t* row_csr = reinterpret_cast<int32_t*>(scr);
  void* scan_tmp = scr + (std::max<int64_t>(R, 1) * 4 + 255) / 256 * 256;
  SHIRO_TRY(scan_generic(SegLen{sg.seg_begin, sg.seg_end}, R, OutPtr{rb.ptr}, rb.ptr + R, scan_tmp, s));
  if (nnz > 0 && R > 0) {
    k_rb_fill<<<grid_for(nnz), kBlock, 0, s>>>(rb.ptr, R, sg.seg_begin, plan->col, nnz, rb.perm, rb.col,
                                                     rb.rid);
    SHIRO_LAUNCH_CHECK();
    if (plan->vmap) SHIRO_TRY(launch_compose(rb.perm, plan->vmap, nnz, s));
    k_rb_agg<<<grid_for(R), kBlock, 0, s>>>(sg.seg_csr, sg.seg_row, R, rb.agg_idx, row_csr, rb.ones);
    SHIRO_LAUNCH_CHECK();
  }
  k_rb_agg_ptr<<<grid_for(rows + 1), kBlock, 0, s>>>(row_csr, R, rows, rb.agg_ptr);
  SHIRO_LAUNCH_CHECK();
  if (R > 0) {
    k_row_ids<<<grid_for(R), kBlock, 0, s>>>(rb.agg_ptr, rows, R, rb.agg_rid);
    SHIRO_LAUNCH_CHECK();
  }
  SHIRO_HIP(hipStreamSynchronize(s));
  rb.built = true;
  return SHIRO_OK;
}

int launch_partial_c(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* B,
                     int64_t ldb, int32_t N, shiro_dtype in_dt, void* Cp, int64_t ldc,
                     shiro_dtype out_dt, hipStream_t s) {
  const RowBased& rb = plan->rb;
  if (rb.R == 0 || N == 0) return SHIRO_OK;
  const bool cap = stream_capturing(s);
  const WorkList* wl;
  SHIRO_TRY(ensure_rb_work(plan, 0, t.chunk, !cap, s, &wl));
  SHIRO_TRY(ensure_carry(plan, (int64_t)wl->W * 2 * N, !cap));
  // values in block-major order (they may change from call to call)
  k_gather_vals<<<grid_for(plan->nnz), kBlock, 0, s>>>(rb.perm, vals + plan->nz_begin, plan->nnz, rb.vals);
  SHIRO_LAUNCH_CHECK();
  return launch_pattern(plan, t, wl, rb.ptr, rb.col, rb.vals, rb.R, B, ldb, N, in_dt, Cp, ldc, out_dt, s,
                        nullptr, rb.rid);
}

int launch_aggregate_c(shiro_plan plan, const shiro_tuning_t& t, const void* Cp, int64_t ldc,
                       int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                       bool accumulate, hipStream_t s) {
  const RowBased& rb = plan->rb;
  if (plan->rows == 0 || N == 0) return SHIRO_OK;
  const bool cap = stream_capturing(s);
  const WorkList* wa;
  SHIRO_TRY(ensure_rb_work(plan, 1, t.chunk, !cap, s, &wa));
  SHIRO_TRY(ensure_carry(plan, (int64_t)wa->W * 2 * N, !cap));
  return launch_pattern(plan, t, wa, rb.agg_ptr, rb.agg_idx, rb.ones, plan->rows, Cp, ldc, N, in_dt, Y, ldy,
                        out_dt, s, accumulate ? rb.iota : nullptr, rb.agg_rid);
}

int launch_spmm_t(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* dY,
                  int64_t lddy, int32_t N, shiro_dtype dt, void* dBp, int64_t lddbp, void* dB,
                  int64_t lddb, bool db_overwrite, const void* Bp, int64_t ldp, float* dvals,
                  bool* dvals_done, hipStream_t s) {
  if (dvals_done) *dvals_done = false;
  if (plan->U == 0 || N == 0 || (!dBp && !dB)) return SHIRO_OK;
  const bool cap = stream_capturing(s);
  if (!plan->tr.built) {
    if (cap) return set_error(SHIRO_ERR_CAPTURING, "backward: transposed pattern not prepared before capture");
    SHIRO_TRY(build_transposed(plan, s));
  }
  const WorkList* wl;
  SHIRO_TRY(ensure_cols_work(plan, t.chunk, !cap, s, &wl));
  SHIRO_TRY(ensure_carry(plan, (int64_t)wl->W * 2 * N, !cap));
  SHIRO_TRY(ensure_tvals(plan, !cap));
  // values in transposed order: one streaming gather per call, so the hot
  // loop reads them contiguously instead of through a dependent index
  k_gather_vals<<<grid_for(plan->nnz), kBlock, 0, s>>>(plan->tr.perm, vals + plan->nz_begin, plan->nnz,
                                                        plan->tvals);
  SHIRO_LAUNCH_CHECK();
  const HotRows* hot = nullptr;
  if (t.group_rows == 3 && t.lds_rows > 0)
    SHIRO_TRY(ensure_hot(plan, SHIRO_KERNEL_SPMM_T, t.lds_rows, !cap, s, &hot));
  SpmmArgs a{};
  a.ptr = plan->tr.ptr;
  a.idx = hot ? hot->walk_idx : plan->tr.row;
  a.hot_src = hot ? hot->hot_src : nullptr;
  a.n_hot = hot ? hot->H : 0;
  a.rid = plan->tr.rid;
  a.vals = plan->tvals;
  a.X = dY;
  a.ldx = lddy;
  a.out = dBp;
  a.ldo = lddbp;
  a.scat = dB;
  a.lds = lddb;
  a.scat_mode = db_overwrite ? 2 : 1;
  a.scat_idx = plan->unique_cols;
  a.chunk_row = wl->chunk_row;
  a.chunk_nz = wl->chunk_nz;
  a.carry = plan->carry;
  a.W = wl->W;
  a.R = (int32_t)plan->U;
  a.N = N;
  int v;
  if (dt == SHIRO_F32) v = vec_for<float>(N, {{dY, lddy}, {dBp, lddbp}, {dB, lddb}, {Bp, ldp}});
  else v = vec_for<bf16_t>(N, {{dY, lddy}, {dBp, lddbp}, {dB, lddb}, {Bp, ldp}});
  // dvals ride along when one column tile covers N
  const bool fuse = dvals && Bp && (int64_t)effective_lanes(64, N, v) * v >= N;
  if (fuse) {
    shiro_tuning_t tt = t;
    tt.lanes = 64;  // one tile (effective lanes then cover N)
    a.D = Bp;
    a.ldd = ldp;
    a.dot_out = plan->tdvals;
    if (dt == SHIRO_F32) SHIRO_TRY((run_spmm_family<float, float>(plan, tt, wl, a, v, s)));
    else SHIRO_TRY((run_spmm_family<bf16_t, bf16_t>(plan, tt, wl, a, v, s)));
    k_scatter_vals<<<grid_for(plan->nnz), kBlock, 0, s>>>(plan->tr.perm, plan->tdvals, plan->nnz,
                                                                     dvals + plan->nz_begin);
    SHIRO_LAUNCH_CHECK();
    if (dvals_done) *dvals_done = true;
    return SHIRO_OK;
  }
  if (dt == SHIRO_F32) return run_spmm_family<float, float>(plan, t, wl, a, v, s);
  return run_spmm_family<bf16_t, bf16_t>(plan, t, wl, a, v, s);
}

int launch_sddmm(shiro_plan plan, const shiro_tuning_t& t, const float*, const void* dY,
                 int64_t lddy, const void* Bp, int64_t ldp, int32_t N, shiro_dtype dt,
                 float* dvals, hipStream_t s) {
  if (plan->nnz == 0) return SHIRO_OK;
  const WorkList* wl;
  SHIRO_TRY(ensure_rows_work(plan, t.chunk, !stream_capturing(s), s, &wl));
  SddmmArgs a{};
  a.ptr = plan->row_ptr;
  a.idx = plan->colmap;
  a.dY = dY;
  a.lddy = lddy;
  a.Bp = Bp;
  a.ldp = ldp;
  a.dvals = dvals + plan->nz_begin;
  a.out_map = plan->vmap;  // subset plans write through the value map
  a.chunk_row = wl->chunk_row;
  a.chunk_nz = wl->chunk_nz;
  a.W = wl->W;
  a.R = (int32_t)plan->rows;
  a.N = N;
  a.xcd_remap = t.xcd_remap;
  shiro_tuning_t tt = t;
  unsigned nb;
  if (dt == SHIRO_F32) {
    const int v = vec_for<float>(N, {{dY, lddy}, {Bp, ldp}});
    tt.lanes = effective_lanes(t.lanes, N, v);
    SHIRO_TRY(grid_waves(plan, tt, wl->W, kWavesPerBlock, &a.chunks_per_wave, &nb));
    if (v == 4) return sddmm_dispatch<float, 4>(tt, dim3(nb), s, a);
    return sddmm_dispatch<float, 1>(tt, dim3(nb), s, a);
  }
  const int v = vec_for<bf16_t>(N, {{dY, lddy}, {Bp, ldp}});
  tt.lanes = effective_lanes(t.lanes, N, v);
  SHIRO_TRY(grid_waves(plan, tt, wl->W, kWavesPerBlock, &a.chunks_per_wave, &nb));
  if (v == 8) return sddmm_dispatch<bf16_t, 8>(tt, dim3(nb), s, a);
  return sddmm_dispatch<bf16_t, 1>(tt, dim3(nb), s, a);
}

// Per-block structures (setup): each column block's own CSR over its (row,
// block) entries, rebased, with a merge-path work list whose chunk size
// spreads the block over the whole persistent grid of the walk.
int build_per_block(shiro_plan plan, hipStream_t s) {
  PerBlock& pb = plan->pb;
  if (pb.built) return SHIRO_OK;
  SHIRO_TRY(build_rowbased(plan, s));
  const RowBased& rb = plan->rb;
  const int64_t R = rb.R, nnz = plan->nnz;
  const int32_t P = plan->P;
  const auto& off = plan->seg.h_off;
  SHIRO_TRY(dev_alloc_n(&pb.ptr, R + P));
  SHIRO_TRY(dev_alloc_n(&pb.idx, std::max<int64_t>(nnz, 1)));
  SHIRO_TRY(dev_alloc_n(&pb.rid, std::max<int64_t>(nnz, 1)));
  k_pb_ptr<<<grid_for(R + P), kBlock, 0, s>>>(rb.ptr, rb.block_off, P, R + P, pb.ptr);
  SHIRO_LAUNCH_CHECK();
  if (nnz > 0) {
    k_pb_fill<<<grid_for(nnz), kBlock, 0, s>>>(rb.rid, rb.perm, plan->colmap, rb.block_off, P, nnz, pb.idx, pb.rid);
    SHIRO_LAUNCH_CHECK();
  }
  std::vector<int64_t> h_ptr((size_t)R + 1);
  SHIRO_HIP(hipMemcpyAsync(h_ptr.data(), rb.ptr, (size_t)(R + 1) * 8, hipMemcpyDeviceToHost, s));
  SHIRO_HIP(hipStreamSynchronize(s));
  const shiro_tuning_t t = tuning_for(plan, SHIRO_KERNEL_SPMM, 128, SHIRO_F32);
  const int64_t workers = (int64_t)plan->num_cus * t.wg_per_cu * kWavesPerBlock * 2;
  pb.work.assign((size_t)P, WorkList{});
  for (int32_t q = 0; q < P; ++q) {
    const int64_t Rq = off[q + 1] - off[q];
    const int64_t nq = h_ptr[off[q + 1]] - h_ptr[off[q]];
    if (nq == 0) continue;
    const int32_t chunk = (int32_t)std::min<int64_t>(std::max<int64_t>(ceil_div(Rq + nq, workers), 16), 4096);
    SHIRO_TRY(build_worklist(pb.ptr + off[q] + q, Rq, nq, chunk, &pb.work[q], s));
    pb.max_W = std::max(pb.max_W, pb.work[q].W);
  }
  pb.nz_off.assign((size_t)P + 1, 0);
  for (int32_t q = 0; q <= P; ++q) pb.nz_off[q] = h_ptr[off[q]];
  pb.built = true;
  return SHIRO_OK;
}

// One launch of the tuned walk per column block, each over that block's own
// work list, adding the block's partial rows into Y in block order (the
// paper's one local product per block followed by aggregation).  Partial
// sums go straight into Y when Y is float32, else into a float32 workspace
// rounded to bfloat16 once at the end.
int launch_spmm_per_block(shiro_plan plan, const float* vals, const void* X, int64_t ldx,
                          int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                          hipStream_t s) {
  if (plan->vmap) return set_error(SHIRO_ERR_UNSUPPORTED, "per-block mode is not available on subset plans");
  if (plan->rows == 0 || N == 0) return SHIRO_OK;
  if (in_dt == SHIRO_F32 && out_dt != SHIRO_F32)
    return set_error(SHIRO_ERR_UNSUPPORTED, "spmm: dtype pair not supported");
  const bool cap = stream_capturing(s);
  if (!plan->pb.built) {
    if (cap) return set_error(SHIRO_ERR_CAPTURING, "per-block spmm: block structures not prepared before capture");
    SHIRO_TRY(build_per_block(plan, s));
  }
  const PerBlock& pb = plan->pb;
  SHIRO_TRY(ensure_carry(plan, (int64_t)pb.max_W * 2 * N, !cap));
  float* acc = reinterpret_cast<float*>(Y);
  int64_t lda = ldy;
  if (out_dt == SHIRO_BF16) {
    SHIRO_TRY(ensure_acc32(plan, plan->rows * (int64_t)N, !cap));
    acc = plan->acc32;
    lda = N;
  }
  k_zero_rows<float><<<grid_for(plan->rows * (int64_t)N, 65536), kBlock, 0, s>>>(acc, plan->rows, lda, N);
  SHIRO_LAUNCH_CHECK();
  if (plan->nnz > 0) {
    // values in block-major order (they may change from call to call)
    k_gather_vals<<<grid_for(plan->nnz), kBlock, 0, s>>>(plan->rb.perm, vals + plan->nz_begin, plan->nnz,
                                                          plan->rb.vals);
    SHIRO_LAUNCH_CHECK();
  }
  shiro_tuning_t t = tuning_for(plan, SHIRO_KERNEL_SPMM, N, in_dt);
  if (t.group_rows < 2) t.group_rows = 2;  // the walk: every block's entries are non-empty rows
  t.lds_rows = 0;                          // the blocks index Bpacked through their own copies
  const auto& off = plan->seg.h_off;
  for (int32_t q = 0; q < plan->P; ++q) {
    const WorkList& wl = pb.work[q];
    if (wl.W == 0) continue;
    const int64_t e0 = off[q], n0 = pb.nz_off[q];
    SpmmArgs a{};
    a.ptr = pb.ptr + e0 + q;
    a.idx = pb.idx + n0;
    a.rid = pb.rid + n0;
    a.vals = plan->rb.vals + n0;
    a.X = X;
    a.ldx = ldx;
    a.scat = acc;
    a.lds = lda;
    a.scat_idx = plan->seg.seg_row + e0;
    a.scat_mode = 1;
    a.chunk_row = wl.chunk_row;
    a.chunk_nz = wl.chunk_nz;
    a.carry = plan->carry;
    a.W = wl.W;
    a.R = (int32_t)(off[q + 1] - e0);
    a.N = N;
    if (in_dt == SHIRO_F32) {
      SHIRO_TRY((run_spmm_family<float, float>(plan, t, &wl, a, vec_for<float>(N, {{X, ldx}, {acc, lda}}), s)));
    } else {
      const int v = vec_for<bf16_t>(N, {{X, ldx}}) == 8 && aligned16<float>(acc, lda) ? 8 : 1;
      SHIRO_TRY((run_spmm_family<bf16_t, float>(plan, t, &wl, a, v, s)));
    }
  }
  if (out_dt == SHIRO_BF16) {
    k_round_rows<<<grid_for(plan->rows * (int64_t)N, 65536), kBlock, 0, s>>>(acc, lda, (bf16_t*)Y, ldy,
                                                                             plan->rows, N);
    SHIRO_LAUNCH_CHECK();
  }
  return SHIRO_OK;
}

int launch_fill_random(float* p, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return SHIRO_OK;
  k_fill_random_f32<<<grid_for(n), kBlock, 0, s>>>(p, n, seed);
  SHIRO_LAUNCH_CHECK();
  return SHIRO_OK;
}

}  // namespace shiro
