// Binning and sorting of (tile | depth, record) entries.
//
//   duplicate   one entry per tile of each record's tile rectangle, written at
//               the record's exclusive-scan offset.  A wavefront owns 64
//               consecutive records, whose entries are contiguous; each lane
//               finds the record of an output slot by binary search over the
//               64 offsets, so writes are coalesced and a record covering
//               thousands of tiles is spread over the whole wavefront.
//   radix sort  stable LSD sort of the 64-bit keys with 8-bit digits, only
//               over the bits in use (32 depth bits + enough tile bits).  One
//               histogram pass computes the digit counts of every pass; each
//               pass is then a single sweep (Onesweep, Adinets & Merrill
//               2022): a block takes a partition ticket, ranks its keys with
//               wave64 ballot match masks, publishes per-digit counts and
//               resolves its global digit offsets by decoupled look-back over
//               the preceding partitions (Merrill & Garland 2016), then
//               scatters through LDS so that global writes are runs of equal
//               digits.
//   ranges      [start, end) of every tile in the sorted order.
//
// The device-side entry count decides all work; the launch grids are sized
// by the caller's capacity, and surplus blocks exit at once.

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kPart = kBlock * kItems;  // keys per partition
constexpr int kRadix = 256;
constexpr int kWaves = kBlock / 64;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;

__device__ __forceinline__ uint64_t entry_count(const uint64_t* n_dup, int64_t capacity) {
  const uint64_t n = *n_dup;
  return n > (uint64_t)capacity ? 0ull : n;
}

__device__ __forceinline__ uint64_t ld_acquire(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_release(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sort_init_kernel(uint32_t* __restrict__ hist, int hist_words,
                                                           uint32_t* __restrict__ tickets, int passes,
                                                           uint64_t* __restrict__ lookback0,
                                                           int64_t lookback_words) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = t; i < hist_words; i += stride) hist[i] = 0u;
  for (int64_t i = t; i < passes; i += stride) tickets[i] = 0u;
  for (int64_t i = t; i < lookback_words; i += stride) lookback0[i] = 0ull;
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = t; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void duplicate_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ tiles,
    const uint64_t* __restrict__ offsets, const uint64_t* __restrict__ n_dup, int64_t n_rec,
    int64_t n_per_cam, CamPack cp, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
    int64_t capacity, int32_t* __restrict__ overflow) {
  __shared__ uint64_t s_off[kWaves][64];
  __shared__ uint32_t s_base[kWaves][64];   // first global tile of the rect
  __shared__ uint32_t s_w[kWaves][64];      // rect width in tiles
  __shared__ uint32_t s_tx[kWaves][64];     // tiles per row of the camera
  __shared__ uint32_t s_depth[kWaves][64];
  const uint64_t total = *n_dup;
  const bool over = total > (uint64_t)capacity;
  if (blockIdx.x == 0 && threadIdx.x == 0) *overflow = over ? 1 : 0;
  if (over) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r = ((int64_t)blockIdx.x * kWaves + wave) * 64 + lane;
  uint32_t cnt = 0;
  uint64_t off = total;
  if (r < n_rec) {
    cnt = tiles[r];
    off = offsets[r];
  }
  if (cnt > 0) {
    const Record& R = rec[r];
    const int cam = (int)(r / n_per_cam);
    const CamDev& C = cp.cam[cam];
    const int sh = cp.tile_shift;
    const uint32_t tx0 = (R.xr & 0xffffu) >> sh, tx1 = (R.xr >> 16) >> sh;
    const uint32_t ty0 = (R.yr & 0xffffu) >> sh;
    s_base[wave][lane] = C.tile_off + ty0 * (uint32_t)C.tiles_x + tx0;
    s_w[wave][lane] = tx1 - tx0 + 1;
    s_tx[wave][lane] = (uint32_t)C.tiles_x;
    s_depth[wave][lane] = R.depth;
  }
  s_off[wave][lane] = off;
  // wave range [start, end): offsets are non-decreasing in r
  const uint64_t start = __shfl(off, 0, 64);
  uint64_t end = off + cnt;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const uint64_t o = __shfl_xor(end, m, 64);
    end = o > end ? o : end;
  }
  if (r >= n_rec && lane == 0) end = start;  // whole wave past the end
  __syncthreads();
  const uint32_t rbase = (uint32_t)(((int64_t)blockIdx.x * kWaves + wave) * 64);
  for (uint64_t o = start + lane; o < end; o += 64) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1)
      if (s_off[wave][lo + step] <= o) lo += step;
    const uint32_t l = (uint32_t)(o - s_off[wave][lo]);
    const uint32_t w = s_w[wave][lo];
    const uint32_t row = l / w, col = l - row * w;
    const uint32_t tile = s_base[wave][lo] + row * s_tx[wave][lo] + col;
    keys[o] = ((uint64_t)tile << 32) | s_depth[wave][lo];
    vals[o] = rbase + (uint32_t)lo;
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void hist_kernel(const uint64_t* __restrict__ keys,
                                                      const uint64_t* __restrict__ n_dup,
                                                      int64_t capacity, int passes,
                                                      uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[8][kRadix];
  for (int i = threadIdx.x; i < 8 * kRadix; i += kBlock) (&s_h[0][0])[i] = 0u;
  __syncthreads();
  const uint64_t n = entry_count(n_dup, capacity);
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < (int64_t)n; i += stride) {
    const uint64_t k = keys[i];
    for (int p = 0; p < passes; ++p) atomicAdd(&s_h[p][(k >> (8 * p)) & 0xffu], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < passes * kRadix; i += kBlock) {
    const uint32_t v = (&s_h[0][0])[i];
    if (v) atomicAdd(&hist[i], v);
  }
}

// Exclusive scan of each pass's 256 digit counts (one block, thread = digit).
__global__ __launch_bounds__(kRadix) void hist_scan_kernel(uint32_t* __restrict__ hist, int passes) {
  __shared__ uint32_t s[kRadix];
  for (int p = 0; p < passes; ++p) {
    const uint32_t v = hist[p * kRadix + threadIdx.x];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kRadix; off <<= 1) {
      const uint32_t add = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    hist[p * kRadix + threadIdx.x] = s[threadIdx.x] - v;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void onesweep_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout, const uint64_t* __restrict__ n_dup,
    int64_t capacity, int shift, const uint32_t* __restrict__ digit_base,
    uint64_t* __restrict__ lookback, uint64_t* __restrict__ lookback_next,
    uint32_t* __restrict__ ticket) {
  __shared__ uint64_t s_keys[kPart];
  __shared__ uint32_t s_vals[kPart];
  __shared__ uint32_t s_cnt[kWaves][kRadix];
  __shared__ uint32_t s_start[kRadix];
  __shared__ uint64_t s_glob[kRadix];
  __shared__ uint32_t s_scan[kWaves];
  __shared__ uint32_t s_part;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  for (int i = t; i < kWaves * kRadix; i += kBlock) (&s_cnt[0][0])[i] = 0u;
  __syncthreads();
  const uint64_t n = entry_count(n_dup, capacity);
  const uint64_t parts = (n + kPart - 1) / kPart;
  const uint32_t part = s_part;
  if (part >= parts) return;
  lookback_next[(uint64_t)part * kRadix + t] = 0ull;

  const uint64_t base = (uint64_t)part * kPart;
  const uint64_t wbase = base + (uint64_t)wave * 64 * kItems;
  uint64_t key[kItems];
  uint32_t val[kItems];
  uint32_t rank[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
    const bool ok = idx < n;
    key[i] = ok ? kin[idx] : ~0ull;
    val[i] = ok ? vin[idx] : 0u;
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t d = (uint32_t)(key[i] >> shift) & 0xffu;
    uint64_t match = ~0ull;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      match &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t below = __popcll(match & lt_mask);
    const uint32_t same = __popcll(match);
    const uint32_t c = s_cnt[wave][d];
    rank[i] = c + below;
    if (below == same - 1) s_cnt[wave][d] = c + same;
  }
  __syncthreads();
  // thread t owns digit t: prefix over waves, block total
  uint32_t tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    const uint32_t c = s_cnt[w][t];
    s_cnt[w][t] = tot;
    tot += c;
  }
  // block-wide exclusive scan of the digit totals
  uint32_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_scan[wave] = inc;
  // publish this partition's digit count before looking back
  uint64_t* my = lookback + (uint64_t)part * kRadix + t;
  if (part == 0)
    st_release(my, kFlagPrefix | (uint64_t)tot);
  else
    st_release(my, kFlagAgg | (uint64_t)tot);
  __syncthreads();
  uint32_t wpre = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w)
    if (w < wave) wpre += s_scan[w];
  const uint32_t start = wpre + inc - tot;
  s_start[t] = start;
  // decoupled look-back for digit t
  uint64_t excl = 0;
  if (part > 0) {
    int64_t j = (int64_t)part - 1;
    while (true) {
      const uint64_t w = ld_acquire(lookback + (uint64_t)j * kRadix + t);
      const uint64_t flag = w & ~kValueMask;
      if (flag == 0) continue;
      excl += w & kValueMask;
      if (flag == kFlagPrefix) break;
      --j;
    }
    st_release(my, kFlagPrefix | (excl + tot));
  }
  s_glob[t] = (uint64_t)digit_base[t] + excl - start;
  __syncthreads();
  // scatter into LDS in block-sorted order
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t d = (uint32_t)(key[i] >> shift) & 0xffu;
    const uint32_t pos = s_start[d] + s_cnt[wave][d] + rank[i];
    s_keys[pos] = key[i];
    s_vals[pos] = val[i];
  }
  __syncthreads();
  const uint64_t nvalid = (n - base) < (uint64_t)kPart ? (n - base) : (uint64_t)kPart;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const uint32_t p = (uint32_t)(i * kBlock + t);
    if (p < nvalid) {
      const uint64_t k = s_keys[p];
      const uint32_t d = (uint32_t)(k >> shift) & 0xffu;
      const uint64_t dst = s_glob[d] + p;
      kout[dst] = k;
      vout[dst] = s_vals[p];
    }
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void ranges_kernel(const uint64_t* __restrict__ keys,
                                                        const uint64_t* __restrict__ n_dup,
                                                        int64_t capacity,
                                                        uint32_t* __restrict__ ranges) {
  const uint64_t n = entry_count(n_dup, capacity);
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t tile = (uint32_t)(keys[i] >> 32);
  if (i == 0 || (uint32_t)(keys[i - 1] >> 32) != tile) ranges[2 * (uint64_t)tile] = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> 32) != tile)
    ranges[2 * (uint64_t)tile + 1] = (uint32_t)(i + 1);
}

struct SortWs {
  uint64_t* alt_keys;
  uint32_t* alt_vals;
  uint32_t* hist;
  uint32_t* tickets;
  uint64_t* lookback[2];
  int64_t parts;
  size_t bytes;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SortWs carve(void* ws, int64_t capacity, int passes) {
  SortWs w;
  const int64_t parts = (capacity + kPart - 1) / kPart;
  w.parts = parts > 0 ? parts : 1;
  char* p = (char*)ws;
  size_t off = 0;
  w.alt_keys = (uint64_t*)(p + off);
  off += align256((size_t)(capacity > 0 ? capacity : 1) * 8);
  w.alt_vals = (uint32_t*)(p + off);
  off += align256((size_t)(capacity > 0 ? capacity : 1) * 4);
  w.hist = (uint32_t*)(p + off);
  off += align256((size_t)8 * kRadix * 4);
  w.tickets = (uint32_t*)(p + off);
  off += align256((size_t)8 * 4);
  for (int b = 0; b < 2; ++b) {
    w.lookback[b] = (uint64_t*)(p + off);
    off += align256((size_t)w.parts * kRadix * 8);
  }
  (void)passes;
  w.bytes = off;
  return w;
}

}  // namespace

size_t sort_workspace_bytes(int64_t capacity, int passes) { return carve(nullptr, capacity, passes).bytes; }

hipError_t launch_bin_sort(const Record* rec, const uint32_t* tiles, const uint64_t* offsets,
                           const uint64_t* n_dup, int64_t n_rec, int64_t n_per_cam,
                           const CamPack& cp, uint64_t* keys, uint32_t* vals, int64_t capacity,
                           uint32_t* ranges, int32_t* overflow, void* ws, int passes,
                           hipStream_t s) {
  SortWs w = carve(ws, capacity, passes);
  // ping-pong so that the last pass lands in the caller's buffers
  uint64_t* kb[2];
  uint32_t* vb[2];
  if (passes % 2 == 0) {
    kb[0] = keys; vb[0] = vals; kb[1] = w.alt_keys; vb[1] = w.alt_vals;
  } else {
    kb[0] = w.alt_keys; vb[0] = w.alt_vals; kb[1] = keys; vb[1] = vals;
  }
  const int64_t lb_words = w.parts * kRadix;
  {
    const int64_t g = (lb_words + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
    hipLaunchKernelGGL(sort_init_kernel, dim3(grid), dim3(kBlock), 0, s, w.hist, passes * kRadix,
                       w.tickets, passes, w.lookback[0], lb_words);
  }
  {
    const int64_t waves = (n_rec + 63) / 64;
    const int64_t blocks = (waves + kWaves - 1) / kWaves;
    hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(kBlock), 0, s,
                       rec, tiles, offsets, n_dup, n_rec, n_per_cam, cp, kb[0], vb[0], capacity,
                       overflow);
  }
  {
    int64_t g = (capacity + kBlock * 16 - 1) / (kBlock * 16);
    const unsigned grid = (unsigned)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
    hipLaunchKernelGGL(hist_kernel, dim3(grid), dim3(kBlock), 0, s, kb[0], n_dup, capacity, passes,
                       w.hist);
    hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(kRadix), 0, s, w.hist, passes);
  }
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL(onesweep_kernel, dim3((unsigned)w.parts), dim3(kBlock), 0, s, kb[p & 1],
                       vb[p & 1], kb[(p + 1) & 1], vb[(p + 1) & 1], n_dup, capacity, 8 * p,
                       w.hist + p * kRadix, w.lookback[p & 1], w.lookback[(p + 1) & 1],
                       w.tickets + p);
  }
  {
    const int64_t nr = 2 * (int64_t)cp.tiles_total;
    const int64_t g = (nr + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)(g < 1 ? 1 : (g > 4096 ? 4096 : g))), dim3(kBlock),
                       0, s, ranges, nr, 0u);
    const int64_t gk = (capacity + kBlock - 1) / kBlock;
    if (gk > 0)
      hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)gk), dim3(kBlock), 0, s, keys, n_dup, capacity,
                         ranges);
  }
  return hipGetLastError();
}

}  // namespace hgs
