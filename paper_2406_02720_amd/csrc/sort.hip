// Binning and sorting of (tile | depth, record) entries.
//
// The entries must end up ordered by the 64-bit key tile << 32 | depth bits,
// ties by record id: each tile's list holds the records covering it in
// (depth, id) order.
//
// Default path ("placement").  Every entry of a record carries that
// record's depth, so the depth order is established once, on the records:
//
//   1. depth keys of the records (+ their digit histograms), four one-sweep
//      passes -> record slots in (depth, id) order;
//   2. per slot the record's tile rectangle and the bands it meets (a band:
//      whole tile rows of one camera, >= kBandTiles tiles); one (band, slot)
//      pair per band met, radix-sorted by band (stable, so each band's slots
//      stay in depth order); each band's pairs are cut into items of
//      kBlockPairs;
//   3. per item, how many of its records cover each tile of the band (LDS
//      difference arrays) -> counts[item][tile]; per tile the total over the
//      items and its exclusive scan over tiles (the tile's range), and per
//      item the position of its first entry of each tile;
//   4. per item a workgroup places the entries: per-wavefront counts,
//      cursors from scans across the wavefronts, each wavefront walks its
//      records in order and takes each covered tile's next slot, so a tile's
//      slots follow (depth, id) order; the slots live in an LDS staging area
//      whose per-tile runs are then copied out in contiguous bursts.
//
// The result is exactly the sorted entry list, at one 4-byte write per entry
// (its record id) instead of a duplication and ceil(tile bits / 8) sorting
// passes over 8-byte pairs.  With HGS_FLAG_SORT_FULL_KEYS the entries are
// instead duplicated with full 64-bit keys in record order and sorted over
// all 32 + tile bits, the literal form of the method's sort; both paths
// produce the same order.
//
// One-sweep pass (Onesweep, Adinets & Merrill 2022): a block takes a
// partition ticket (forward progress: earlier partitions belong to blocks
// already running), ranks its keys within each wavefront with wave64 ballot
// match masks, publishes per-digit counts and resolves its global digit
// offsets by decoupled look-back over the preceding partitions (Merrill &
// Garland 2016), then scatters through LDS so that global writes are runs of
// equal digits.  Histograms use the same ballot match so that a wavefront
// adds each distinct digit once.
//
// The device-side counts decide all work; grids are sized from bounds (the
// caller's capacity, the pair bound) and the kernels whose true work can be
// much smaller loop over it from a bounded grid (one-sweep partitions by
// ticket, placement items by stride).

#include "hgs_internal.h"

namespace hgs {

namespace {

constexpr int kBlock = 256;
constexpr int kRadix = 256;
// keys per thread of a one-sweep pass: 32-bit keys use 8192-key partitions,
// 64-bit keys 4096 (LDS holds a partition's keys and values)
template <typename K>
struct SweepItems {
  static constexpr int value = sizeof(K) == 4 ? 32 : 16;
};
// the record, pair and tile-order sorts (a few million keys at most) use
// 4096-key partitions: a million records make 245 of them, about one per
// CU, and the look-back chains stay short (2048-key partitions measured
// 25 us slower over the five passes of a step, 1024-key ones slower still)
constexpr int kSmallItems = 16;
constexpr int kPartMinEntries = kBlock * 16;          // smallest entry partition
constexpr int kPartMinSmall = kBlock * kSmallItems;   // record / tile-order partition
// Digit histograms are accumulated in kHistCopies replicas (block b adds to
// replica b % kHistCopies): thousands of blocks adding to one 256-word
// histogram serialise on a few cache lines.
constexpr int kHistCopies = 128;
constexpr int kWaves = kBlock / 64;
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr int kLookWindow = 8;   // look-back flags requested per round trip
constexpr int kMaxPasses = 8;
constexpr int kHistWords = 2 * kMaxPasses * kRadix;  // one replica: record + entry passes

__device__ __forceinline__ uint64_t entry_count(const uint64_t* n_dev, int64_t capacity) {
  if (!n_dev) return (uint64_t)capacity;
  const uint64_t n = *n_dev;
  return n > (uint64_t)capacity ? 0ull : n;
}

__device__ __forceinline__ uint64_t ld_flag(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Lanes of the wavefront holding the same 8-bit digit as this lane (all 64
// lanes must call).
__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bal = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bal : ~bal;
  }
  return m;
}

// bins[d] += 1 for every valid lane, one LDS atomic per distinct digit.
__device__ __forceinline__ void wave_hist_add(uint32_t* bins, uint32_t d, bool valid) {
  const uint64_t m = match_digit(d) & __ballot(valid);
  if (valid && (int)__lane_id() == __ffsll((unsigned long long)m) - 1)
    atomicAdd(&bins[d], (uint32_t)__popcll(m));
}

__device__ __forceinline__ void flush_hist(const uint32_t* s_h, int words, uint32_t* hist) {
  uint32_t* dst = hist + (blockIdx.x % kHistCopies) * kHistWords;
  for (int i = threadIdx.x; i < words; i += blockDim.x) {
    const uint32_t v = s_h[i];
    if (v) atomicAdd(&dst[i], v);
  }
}

// ---------------------------------------------------------------------------
// Clears the digit histograms, the pass tickets, the look-back flags of the
// first one-sweep pass (every pass clears those of the next) and
// (placement path) the band ranges and tile totals, which are only written
// later in the call.
__global__ __launch_bounds__(kBlock) void sort_init_kernel(uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ tickets,
                                                           uint64_t* __restrict__ lookback, int64_t n_lookback,
                                                           uint32_t* __restrict__ brange, int64_t n_brange,
                                                           uint32_t* __restrict__ totals, int64_t n_totals) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = t; i < (int64_t)kHistCopies * kHistWords; i += stride) hist[i] = 0u;
  for (int64_t i = t; i < 2 * kMaxPasses; i += stride) tickets[i] = 0u;
  for (int64_t i = t; i < n_lookback; i += stride) lookback[i] = 0ull;
  for (int64_t i = t; i < n_brange; i += stride) brange[i] = 0u;
  for (int64_t i = t; i < n_totals; i += stride) totals[i] = 0u;
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = t; i < n; i += stride) p[i] = v;
}

// Sum of the replicas and exclusive scan of each pass's 256 digit counts
// (one block of kHistScanThreads: each digit's replicas are summed by four
// threads, 32 replicas each, then one thread per digit scans); `hist` points
// at the passes of replica 0, `bases` receives the scans.
constexpr int kHistScanThreads = 4 * kRadix;
static_assert(kHistCopies % 4 == 0, "four threads per digit");

__global__ __launch_bounds__(kHistScanThreads) void hist_scan_kernel(const uint32_t* __restrict__ hist,
                                                                     uint32_t* __restrict__ bases, int passes) {
  __shared__ uint32_t s_part[4][kRadix];
  __shared__ uint32_t s_wave[kRadix / 64];
  const int t = threadIdx.x, d = t & (kRadix - 1), q = t >> 8;
  constexpr int kPer = kHistCopies / 4;
  // every pass's histograms are read before the first base is stored: the
  // vector memory counter orders loads and stores, so a pass's loads issued
  // after the previous pass's stores would wait for them
  uint32_t vp[kMaxPasses];
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) {
    uint32_t v = 0;
    if (p < passes) {
      const uint32_t* h = hist + (size_t)q * kPer * kHistWords + p * kRadix + d;
#pragma unroll 16
      for (int c = 0; c < kPer; ++c) v += h[(size_t)c * kHistWords];
    }
    vp[p] = v;
  }
#pragma unroll
  for (int p = 0; p < kMaxPasses; ++p) {
    if (p >= passes) break;
    s_part[q][d] = vp[p];
    __syncthreads();
    // threads below kRadix (whole wavefronts) own a digit each
    const int lane = t & 63, wv = t >> 6;
    uint32_t x = 0, inc = 0;
    if (t < kRadix) {
      x = s_part[0][d] + s_part[1][d] + s_part[2][d] + s_part[3][d];
      inc = x;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(inc, off, 64);
        if (lane >= off) inc += y;
      }
      if (lane == 63) s_wave[wv] = inc;
    }
    __syncthreads();
    if (t < kRadix) {
      uint32_t pre = 0;
      for (int w = 0; w < wv; ++w) pre += s_wave[w];
      bases[p * kRadix + d] = pre + inc - x;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// depth-first path
// ---------------------------------------------------------------------------
// Depth key of every record (culled records sort last and emit nothing) and
// the histograms of its four digits; also each record's tile rectangle in
// record order (tx0 | w << 16, ty0 | ty1 << 16; w = 0 for a culled record):
// the depth-order gather of the rectangles then reads this compact array
// instead of whole records.
__global__ __launch_bounds__(kBlock) void depth_keys_kernel(const Record* __restrict__ rec,
                                                            const uint32_t* __restrict__ tiles,
                                                            int64_t n_rec, uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ ids,
                                                            uint32_t* __restrict__ hist,
                                                            uint2* __restrict__ rects, int sh) {
  __shared__ uint32_t s_h[4 * kRadix];
  for (int i = threadIdx.x; i < 4 * kRadix; i += kBlock) s_h[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n_rec; base += stride) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < n_rec;
    uint32_t k = 0xffffffffu;
    if (ok) {
      const bool vis = tiles[i] != 0u;
      // the record's last 16 bytes: rect x, rect y, depth bits, tiles
      const uint4 q = reinterpret_cast<const uint4*>(rec + i)[3];
      k = vis ? q.z : 0xffffffffu;
      keys[i] = k;
      ids[i] = (uint32_t)i;
      const uint32_t tx0 = (q.x & 0xffffu) >> sh, tx1 = (q.x >> 16) >> sh;
      const uint32_t ty0 = (q.y & 0xffffu) >> sh, ty1 = (q.y >> 16) >> sh;
      rects[i] = vis ? make_uint2(tx0 | ((tx1 - tx0 + 1) << 16), ty0 | (ty1 << 16)) : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) wave_hist_add(s_h + p * kRadix, (k >> (8 * p)) & 0xffu, ok);
  }
  __syncthreads();
  flush_hist(s_h, 4 * kRadix, hist);
}

// Output chunks of the duplication: a wavefront writes the entries
// [c * kChunk, (c + 1) * kChunk).  Balancing by output rather than by record
// matters because, in depth order, the nearest kernels -- the ones covering
// the most tiles -- are adjacent.
constexpr int kChunk = 2048;

// chunk_start[c] = the slot whose entries contain position c * kChunk, for
// the n_chunks chunks that fit the capacity (entries beyond it are never
// written: the duplication reports the overflow instead).
__global__ __launch_bounds__(kBlock) void chunk_start_kernel(const uint32_t* __restrict__ order,
                                                             const uint32_t* __restrict__ tiles,
                                                             const uint64_t* __restrict__ offsets,
                                                             int64_t n_rec, uint64_t n_chunks,
                                                             uint32_t* __restrict__ chunk_start) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n_rec) return;
  const uint32_t cnt = tiles[order ? order[j] : (uint32_t)j];
  if (cnt == 0) return;
  const uint64_t a = offsets[j], b = a + cnt;
  for (uint64_t c = (a + kChunk - 1) / kChunk; c * kChunk < b && c < n_chunks; ++c)
    chunk_start[c] = (uint32_t)j;
}

// One entry per covered tile, for the record slots in `order` (identity when
// null) whose entries start at `offsets`.  The wavefront of chunk c loads the
// descriptors of 64 consecutive slots (from chunk_start[c]) into LDS and
// emits the chunk's entries that fall in them, 64 at a time; each lane finds
// the slot of its output position by binary search over the 64 offsets, so
// writes are coalesced and a kernel covering many tiles is spread over many
// lanes and wavefronts.  KEY64 writes tile << 32 | depth keys, otherwise
// 32-bit tile keys; `hist` receives the digit histograms of the key bits
// from `hist_shift` on, `hist_passes` digits.
template <bool KEY64>
__global__ __launch_bounds__(kBlock) void duplicate_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ order,
    const uint32_t* __restrict__ tiles, const uint64_t* __restrict__ offsets,
    const uint32_t* __restrict__ chunk_start, const uint64_t* __restrict__ n_dup, int64_t n_rec,
    int64_t n_per_cam, CamPack cp, void* __restrict__ keys_out, uint32_t* __restrict__ vals,
    int64_t capacity, int32_t* __restrict__ overflow, uint32_t* __restrict__ hist, int hist_shift,
    int hist_passes) {
  __shared__ uint64_t s_off[kWaves][64];
  __shared__ uint32_t s_base[kWaves][64];   // first global tile of the rect
  __shared__ uint32_t s_w[kWaves][64];      // rect width in tiles
  __shared__ uint32_t s_tx[kWaves][64];     // tiles per row of the camera
  __shared__ uint32_t s_depth[kWaves][64];
  __shared__ uint32_t s_id[kWaves][64];
  __shared__ uint32_t s_h[kMaxPasses * kRadix];
  for (int i = threadIdx.x; i < hist_passes * kRadix; i += kBlock) s_h[i] = 0u;
  __syncthreads();
  const uint64_t total = *n_dup;
  const bool over = total > (uint64_t)capacity;
  if (blockIdx.x == 0 && threadIdx.x == 0) *overflow = over ? 1 : 0;
  if (over) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t c = (uint64_t)blockIdx.x * kWaves + wave;
  const uint64_t o_begin = c * kChunk;
  const uint64_t o_end = o_begin + kChunk < total ? o_begin + kChunk : total;
  if (o_begin < total) {
    int64_t j0 = chunk_start[c];
    while (true) {
      // descriptors of slots j0 .. j0 + 63
      const int64_t j = j0 + lane;
      uint32_t cnt = 0;
      uint64_t off = total;
      if (j < n_rec) {
        const uint32_t r = order ? order[j] : (uint32_t)j;
        cnt = tiles[r];
        off = offsets[j];
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
          s_id[wave][lane] = r;
        }
      }
      s_off[wave][lane] = off;
      uint64_t win_end = off + cnt;  // end of the window's entries (max over lanes)
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) {
        const uint64_t o = __shfl_xor(win_end, m, 64);
        win_end = o > win_end ? o : win_end;
      }
      const uint64_t win_begin = __shfl(off, 0, 64);
      const uint64_t lo_o = win_begin > o_begin ? win_begin : o_begin;
      const uint64_t hi_o = win_end < o_end ? win_end : o_end;
      for (uint64_t o0 = lo_o; o0 < hi_o; o0 += 64) {
        const uint64_t o = o0 + lane;
        const bool ok = o < hi_o;
        uint32_t tile = 0;
        if (ok) {
          int lo = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1)
            if (s_off[wave][lo + step] <= o) lo += step;
          const uint32_t l = (uint32_t)(o - s_off[wave][lo]);
          const uint32_t w = s_w[wave][lo];
          const uint32_t row = l / w, col = l - row * w;
          tile = s_base[wave][lo] + row * s_tx[wave][lo] + col;
          if (KEY64)
            static_cast<uint64_t*>(keys_out)[o] = ((uint64_t)tile << 32) | s_depth[wave][lo];
          else
            static_cast<uint32_t*>(keys_out)[o] = tile;
          vals[o] = s_id[wave][lo];
        }
        for (int p = 0; p < hist_passes; ++p) {
          const int sh = hist_shift + 8 * p;
          const uint32_t d = KEY64 ? (uint32_t)((((uint64_t)tile << 32) >> sh) & 0xffu)
                                   : ((tile >> sh) & 0xffu);
          wave_hist_add(s_h + p * kRadix, d, ok);
        }
      }
      if (win_end >= o_end || j0 + 64 >= n_rec) break;
      j0 += 64;
    }
  }
  __syncthreads();
  flush_hist(s_h, hist_passes * kRadix, hist);
}

// Histogram of the depth digits of 64-bit entries (full-key path): every
// entry of a record has the record's depth, so each record adds its tile
// count to its depth digits.
__global__ __launch_bounds__(kBlock) void depth_hist_weighted_kernel(const Record* __restrict__ rec,
                                                                     const uint32_t* __restrict__ tiles,
                                                                     int64_t n_rec,
                                                                     uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[4 * kRadix];
  for (int i = threadIdx.x; i < 4 * kRadix; i += kBlock) s_h[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n_rec; i += stride) {
    const uint32_t c = tiles[i];
    if (c) {
      const uint32_t k = rec[i].depth;
#pragma unroll
      for (int p = 0; p < 4; ++p) atomicAdd(&s_h[p * kRadix + ((k >> (8 * p)) & 0xffu)], c);
    }
  }
  __syncthreads();
  flush_hist(s_h, 4 * kRadix, hist);
}

// ---------------------------------------------------------------------------
// Persistent one-sweep workgroups: as many as the chip holds at once (about
// 39 KB of LDS each: four per CU).  More only queue behind the resident ones
// and, when the partitions are fewer than the grid (the pair pass is sized
// for its largest count), take an empty ticket after those are done.
constexpr int64_t kSweepGrid = 1024;

template <typename K, int ITEMS>
__global__ __launch_bounds__(kBlock) void onesweep_kernel(
    const K* __restrict__ kin, const uint32_t* __restrict__ vin, K* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint64_t* __restrict__ n_dev, int64_t capacity, int shift,
    const uint32_t* __restrict__ digit_base, uint64_t* __restrict__ lookback,
    uint64_t* __restrict__ lookback_next, int64_t n_lookback, uint32_t* __restrict__ ticket) {
  constexpr int PART = kBlock * ITEMS;
  __shared__ K s_keys[PART];
  __shared__ uint32_t s_vals[PART];
  __shared__ uint32_t s_cnt[kWaves][kRadix];
  __shared__ uint32_t s_start[kRadix];
  __shared__ uint64_t s_glob[kRadix];
  __shared__ uint32_t s_scan[kWaves];
  __shared__ uint32_t s_part;

  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const uint64_t n = entry_count(n_dev, capacity);
  const uint64_t parts = (n + PART - 1) / PART;
  // persistent: partitions are taken by ticket until none is left (a
  // partition's look-back only waits on lower tickets, held by running
  // workgroups)
  for (;;) {
  if (t == 0) s_part = atomicAdd(ticket, 1u);
  for (int i = t; i < kWaves * kRadix; i += kBlock) (&s_cnt[0][0])[i] = 0u;
  __syncthreads();
  const uint32_t part = s_part;
  if (part >= parts) break;

  const uint64_t base = (uint64_t)part * PART;
  const uint64_t wbase = base + (uint64_t)wave * 64 * ITEMS;
  K key[ITEMS];
  uint32_t val[ITEMS];
  uint32_t rank[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint64_t idx = wbase + (uint64_t)i * 64 + lane;
    const bool ok = idx < n;
    key[i] = ok ? kin[idx] : (K)~(K)0;
    val[i] = ok ? vin[idx] : 0u;
  }
  // rank within the wavefront, in item-then-lane order (stable)
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t d = (uint32_t)(key[i] >> shift) & 0xffu;
    const uint64_t match = match_digit(d);
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
  // publish this partition's digit count as early as possible
  uint64_t* my = lookback + (uint64_t)part * kRadix + t;
  st_flag(my, (part == 0 ? kFlagPrefix : kFlagAgg) | (uint64_t)tot);
  uint32_t inc = tot;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  if (lane == 63) s_scan[wave] = inc;
  __syncthreads();
  uint32_t wpre = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w)
    if (w < wave) wpre += s_scan[w];
  const uint32_t start = wpre + inc - tot;
  s_start[t] = start;
  __syncthreads();
  // scatter into LDS in block-sorted order (needs only block-local offsets,
  // so it runs before the look-back and hides part of its latency)
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t d = (uint32_t)(key[i] >> shift) & 0xffu;
    const uint32_t pos = s_start[d] + s_cnt[wave][d] + rank[i];
    s_keys[pos] = key[i];
    s_vals[pos] = val[i];
  }
  // decoupled look-back for digit t, kLookWindow predecessors per round
  // trip: their flags are requested together, then taken in order until an
  // inclusive prefix (done), an unpublished one (wait, then read again from
  // it) or the end of the window (the next window).  Partition 0 always
  // holds a prefix, and a read below it counts as an empty prefix, so the
  // walk ends.
  uint64_t excl = 0;
  if (part > 0) {
    int64_t j = (int64_t)part - 1;
    while (true) {
      uint64_t w[kLookWindow];
#pragma unroll
      for (int q = 0; q < kLookWindow; ++q)
        w[q] = j - q >= 0 ? ld_flag(lookback + (uint64_t)(j - q) * kRadix + t) : kFlagPrefix;
      int used = kLookWindow;
      bool done = false;
#pragma unroll
      for (int q = 0; q < kLookWindow; ++q) {
        const uint64_t flag = w[q] & ~kValueMask;
        if (flag == 0) {
          used = q;
          break;
        }
        excl += w[q] & kValueMask;
        if (flag == kFlagPrefix) {
          done = true;
          break;
        }
      }
      if (done) break;
      j -= used;
      if (used != kLookWindow) __builtin_amdgcn_s_sleep(1);
    }
    st_flag(my, kFlagPrefix | (excl + tot));
  }
  s_glob[t] = (uint64_t)digit_base[t] + excl - start;
  __syncthreads();
  const uint64_t nvalid = (n - base) < (uint64_t)PART ? (n - base) : (uint64_t)PART;
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t p = (uint32_t)(i * kBlock + t);
    if (p < nvalid) {
      const K k = s_keys[p];
      const uint32_t d = (uint32_t)(k >> shift) & 0xffu;
      const uint64_t dst = s_glob[d] + p;
      kout[dst] = k;
      vout[dst] = s_vals[p];
    }
  }
  __syncthreads();
  }
  // the next pass's look-back flags, all of them (whatever its partition
  // count): this pass does not read them and the previous one is done.
  // Cleared last: stores issued before the partitions' loads would make
  // those loads wait for them (the vector memory counter orders both).
  for (int64_t i = (int64_t)blockIdx.x * kBlock + t; i < n_lookback; i += (int64_t)gridDim.x * kBlock)
    lookback_next[i] = 0ull;
}

// ---------------------------------------------------------------------------
template <typename K>
__global__ __launch_bounds__(kBlock) void ranges_kernel(const K* __restrict__ keys, int key_shift,
                                                        const uint64_t* __restrict__ n_dup,
                                                        int64_t capacity,
                                                        uint32_t* __restrict__ ranges) {
  const uint64_t n = entry_count(n_dup, capacity);
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t tile = (uint32_t)(keys[i] >> key_shift);
  if (i == 0 || (uint32_t)(keys[i - 1] >> key_shift) != tile) ranges[2 * (uint64_t)tile] = (uint32_t)i;
  if (i == n - 1 || (uint32_t)(keys[i + 1] >> key_shift) != tile)
    ranges[2 * (uint64_t)tile + 1] = (uint32_t)(i + 1);
}

// Processing order of the tiles, longest list first: 16-bit key
// 0xffff - min(length, 0xffff), value = tile id, and the histograms of its
// two digits.
// Tile order key: the number of entries on a log scale with 4 fractional
// bits (16 buckets per doubling, computed in integers), longest first:
// 255 - min(255, 16 msb(n + 1) + next four bits).  Lists of 2^16 - 1
// entries and more share the first bucket.
__device__ __forceinline__ uint32_t order_key(uint32_t len) {
  const uint32_t v = len + 1u;                 // >= 1
  const int msb = 31 - __clz((int)v);
  const uint32_t frac = (uint32_t)(((uint64_t)v << (32 - msb)) >> 28) & 15u;
  const uint32_t b = (uint32_t)msb * 16u + frac;
  return 255u - (b < 255u ? b : 255u);
}

__global__ __launch_bounds__(kBlock) void order_keys_kernel(const uint32_t* __restrict__ ranges,
                                                            int64_t n_tiles, uint32_t* __restrict__ keys,
                                                            uint32_t* __restrict__ ids,
                                                            uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kRadix];
  for (int i = threadIdx.x; i < kRadix; i += kBlock) s_h[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n_tiles; base += stride) {
    const int64_t t = base + threadIdx.x;
    const bool ok = t < n_tiles;
    uint32_t k = 0;
    if (ok) {
      k = order_key(ranges[2 * t + 1] - ranges[2 * t]);
      keys[t] = k;
      ids[t] = (uint32_t)t;
    }
    wave_hist_add(s_h, k, ok);
  }
  __syncthreads();
  flush_hist(s_h, kRadix, hist);
}

// Optional 64-bit keys of the placed entries: one wavefront per tile writes
// tile << 32 | depth bits over the tile's range.
__global__ __launch_bounds__(64) void keys_from_ranges_kernel(const uint32_t* __restrict__ ranges,
                                                              const uint32_t* __restrict__ vals,
                                                              const Record* __restrict__ rec,
                                                              int64_t n_tiles, uint64_t* __restrict__ keys) {
  const int64_t t = blockIdx.x;
  if (t >= n_tiles) return;
  const uint32_t a = ranges[2 * t], e = ranges[2 * t + 1];
  for (uint32_t p = a + threadIdx.x; p < e; p += 64)
    keys[p] = ((uint64_t)t << 32) | rec[vals[p]].depth;
}

// ---------------------------------------------------------------------------
// placement path
// ---------------------------------------------------------------------------
constexpr int kBandTiles = 256;      // a band: whole tile rows of one camera, >= 256 tiles
constexpr int kItemGroup = 32;       // items per partial sum in the tile scans
constexpr int kBlockPairs = 512;     // (record, band) pairs per placement block
constexpr int64_t kItemGrid = 2048;  // workgroups that loop over the items (their count is on the device)

// Tile rows per band of a camera with `tiles_x` tiles per row.
__host__ __device__ inline int band_rows(int tiles_x) {
  return tiles_x >= kBandTiles ? 1 : kBandTiles / tiles_x;
}

struct PlaceGeom {
  int64_t n_bands;
  int band_tiles;      // largest band (LDS cursors)
  int max_bands;       // most bands of one camera (bound on bands per record)
  int64_t pairs_max;   // bound on (record, band) pairs
  int64_t items_max;   // bound on (band, block) items
  int band_bits;       // bits of a band id
};

PlaceGeom place_geom(int64_t n_rec, int64_t capacity, const CamPack& cp) {
  PlaceGeom g{};
  g.band_tiles = 1;
  for (int c = 0; c < cp.n_cams; ++c) {
    const int tx = cp.cam[c].tiles_x, ty = cp.cam[c].tiles_y, rows = band_rows(tx);
    const int nb = (ty + rows - 1) / rows;
    g.n_bands += nb;
    g.max_bands = nb > g.max_bands ? nb : g.max_bands;
    g.band_tiles = rows * tx > g.band_tiles ? rows * tx : g.band_tiles;
  }
  g.n_bands = g.n_bands > 0 ? g.n_bands : 1;
  // every pair holds at least one entry, and a record meets at most
  // max_bands bands
  const int64_t by_rec = (n_rec > 0 ? n_rec : 0) * (int64_t)(g.max_bands > 0 ? g.max_bands : 1);
  g.pairs_max = capacity < by_rec ? capacity : by_rec;
  g.pairs_max = g.pairs_max > 0 ? g.pairs_max : 1;
  g.items_max = g.n_bands + (g.pairs_max + kBlockPairs - 1) / kBlockPairs;
  g.band_bits = 0;
  while ((1ll << g.band_bits) < g.n_bands) ++g.band_bits;
  return g;
}

struct Band {
  int cam;
  int r0, r1;          // tile rows [r0, r1)
  int tx;              // tiles per row
  uint32_t lo;         // first tile id
  int n;               // tiles in the band
};

// Band k (global numbering: the bands of camera 0, then of camera 1, ...).
__device__ __forceinline__ Band band_of(const CamPack& cp, int64_t k) {
  Band b{};
  for (int c = 0; c < cp.n_cams; ++c) {
    const int tx = cp.cam[c].tiles_x, ty = cp.cam[c].tiles_y, rows = band_rows(tx);
    const int64_t nb = (ty + rows - 1) / rows;
    if (k < nb) {
      b.cam = c;
      b.r0 = (int)k * rows;
      b.r1 = b.r0 + rows < ty ? b.r0 + rows : ty;
      b.tx = tx;
      b.lo = cp.cam[c].tile_off + (uint32_t)(b.r0 * tx);
      b.n = (b.r1 - b.r0) * tx;
      return b;
    }
    k -= nb;
  }
  return b;
}

// First band of camera c and its rows per band.
__device__ __forceinline__ void camera_bands(const CamPack& cp, int c, int64_t* first, int* rows) {
  int64_t f = 0;
  for (int i = 0; i < c; ++i) {
    const int r = band_rows(cp.cam[i].tiles_x);
    f += (cp.cam[i].tiles_y + r - 1) / r;
  }
  *first = f;
  *rows = band_rows(cp.cam[c].tiles_x);
}

__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t x, int lane, uint32_t* total) {
  uint32_t inc = x;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(inc, off, 64);
    if (lane >= off) inc += y;
  }
  *total = __shfl(inc, 63, 64);
  return inc - x;
}

// Per slot j of the depth order: the record's tile rectangle, packed as
// record id, tx0 | w << 16, ty0 | ty1 << 16, camera (from the compact
// rectangles of depth_keys_kernel), and the number of bands it meets.
__global__ __launch_bounds__(kBlock) void place_desc_kernel(const uint2* __restrict__ rects,
                                                            const uint32_t* __restrict__ order, int64_t n_rec,
                                                            int64_t n_per_cam, CamPack cp, uint4* __restrict__ desc,
                                                            uint32_t* __restrict__ nbands) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= n_rec) return;
  const uint32_t r = order[j];
  const uint2 c = rects[r];
  uint32_t nb = 0;
  uint4 d = make_uint4(r, 0u, 0u, 0u);
  if ((c.x >> 16) != 0u) {   // w >= 1: not culled
    const int cam = (int)(r / (uint64_t)n_per_cam);
    d = make_uint4(r, c.x, c.y, (uint32_t)cam);
    const uint32_t rows = (uint32_t)band_rows(cp.cam[cam].tiles_x);
    nb = (d.z >> 16) / rows - (d.z & 0xffffu) / rows + 1;
  }
  desc[j] = d;
  nbands[j] = nb;
}

// (band, slot) pairs in slot order, with the histograms of the band digits.
// Band-count histogram in LDS: bands up to this many take the difference
// array below, more bands the per-pair digit increments.
constexpr int kPairBandsLds = 4096;

__global__ __launch_bounds__(kBlock) void place_pairs_kernel(const uint4* __restrict__ desc,
                                                             const uint32_t* __restrict__ nbands,
                                                             const uint64_t* __restrict__ poff, int64_t n_rec,
                                                             int64_t pairs_max, CamPack cp, int64_t n_bands,
                                                             uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval,
                                                             uint32_t* __restrict__ hist, int hist_passes) {
  __shared__ uint32_t s_h[kMaxPasses * kRadix];
  __shared__ uint32_t s_bd[kPairBandsLds + 1];   // +1 at a record's first band, -1 after its last
  __shared__ uint32_t s_part[kBlock / 64];
  const bool by_band = n_bands <= kPairBandsLds;
  for (int i = threadIdx.x; i < hist_passes * kRadix; i += kBlock) s_h[i] = 0u;
  if (by_band)
    for (int i = threadIdx.x; i <= (int)n_bands; i += kBlock) s_bd[i] = 0u;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t base = (int64_t)blockIdx.x * kBlock; base < n_rec; base += stride) {
    const int64_t j = base + threadIdx.x;
    uint32_t nb = 0, kb0 = 0;
    uint64_t o = 0;
    if (j < n_rec) {
      nb = nbands[j];
      if (nb) {
        const uint4 d = desc[j];
        int64_t first;
        int rows;
        camera_bands(cp, (int)d.w, &first, &rows);
        kb0 = (uint32_t)first + (d.z & 0xffffu) / (uint32_t)rows;
        o = poff[j];
      }
    }
    if (by_band) {
      if (nb) {
        atomicAdd(&s_bd[kb0], 1u);
        atomicSub(&s_bd[kb0 + nb], 1u);
      }
      const bool fits = o + nb <= (uint64_t)pairs_max;  // past the bound only on overflow
      for (uint32_t b = 0; b < nb && fits; ++b) {
        pkey[o + b] = kb0 + b;
        pval[o + b] = (uint32_t)j;
      }
      continue;
    }
    // many bands: the wavefront walks the pairs of its lanes' records
    // together, so the digit histograms see every pair once
    uint32_t most = nb;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      const uint32_t t = __shfl_xor(most, m, 64);
      most = t > most ? t : most;
    }
    for (uint32_t b = 0; b < most; ++b) {
      const bool ok = b < nb && o + b < (uint64_t)pairs_max;
      const uint32_t k = kb0 + b;
      if (ok) {
        pkey[o + b] = k;
        pval[o + b] = (uint32_t)j;
      }
      for (int p = 0; p < hist_passes; ++p) wave_hist_add(s_h + p * kRadix, (k >> (8 * p)) & 0xffu, ok);
    }
  }
  __syncthreads();
  if (by_band) {
    // band counts = prefix sums of the difference array; each band adds
    // its count to its digits' bins
    const int nbd = (int)n_bands;
    const int chunk = (nbd + kBlock - 1) / kBlock;
    const int c0 = threadIdx.x * chunk, c1 = c0 + chunk < nbd ? c0 + chunk : nbd;
    uint32_t run = 0;
    for (int i = c0; i < c1; ++i) run += s_bd[i];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t wtot;
    const uint32_t wex = wave_excl_scan_u32(run, lane, &wtot);
    if (lane == 0) s_part[wv] = wtot;
    __syncthreads();
    uint32_t acc = wex;
    for (int w = 0; w < wv; ++w) acc += s_part[w];
    for (int i = c0; i < c1; ++i) {
      acc += s_bd[i];
      if (acc)
        for (int p = 0; p < hist_passes; ++p) atomicAdd(&s_h[p * kRadix + ((i >> (8 * p)) & 0xff)], acc);
    }
    __syncthreads();
  }
  flush_hist(s_h, hist_passes * kRadix, hist);
}

// [start, end) of every band in the sorted pairs (bands without pairs keep
// the cleared [0, 0)).
__global__ __launch_bounds__(kBlock) void place_band_ranges_kernel(const uint32_t* __restrict__ pkey,
                                                                   const uint64_t* __restrict__ n_pairs,
                                                                   int64_t pairs_max, uint32_t* __restrict__ brange) {
  const uint64_t n = *n_pairs > (uint64_t)pairs_max ? 0ull : *n_pairs;  // more pairs: entries overflow
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t k = pkey[i];
    if (i == 0 || pkey[i - 1] != k) brange[2 * (uint64_t)k] = (uint32_t)i;
    if (i + 1 == n || pkey[i + 1] != k) brange[2 * (uint64_t)k + 1] = (uint32_t)(i + 1);
  }
}

// Blocks of kBlockPairs pairs per band.
__global__ __launch_bounds__(kBlock) void place_band_items_kernel(const uint32_t* __restrict__ brange,
                                                                  int64_t n_bands, uint32_t* __restrict__ nitems) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n_bands) return;
  const uint32_t len = brange[2 * k + 1] - brange[2 * k];
  nitems[k] = (len + kBlockPairs - 1) / kBlockPairs;
}

// item -> band for the items of every band (band k owns items
// [item0[k], item0[k] + nitems[k]), ascending): one thread per item, a
// binary search for the first band whose items end past it (bands without
// items never qualify).
__global__ __launch_bounds__(kBlock) void place_item_bands_kernel(const uint32_t* __restrict__ nitems,
                                                                  const uint64_t* __restrict__ item0,
                                                                  const uint64_t* __restrict__ n_items,
                                                                  int64_t n_bands, uint32_t* __restrict__ item_band) {
  const uint64_t items = *n_items;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < items; i += stride) {
    int64_t lo = 0, hi = n_bands - 1;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (item0[mid] + nitems[mid] > i) hi = mid; else lo = mid + 1;
    }
    item_band[i] = (uint32_t)lo;
  }
}

// counts[item][t] for the tiles t of the item's band: how many of the
// item's records cover t (two LDS increments per rect row into a
// difference array, then its prefix sum).
__global__ __launch_bounds__(64) void place_count_kernel(
    const uint4* __restrict__ desc, const uint32_t* __restrict__ pval, const uint32_t* __restrict__ brange,
    const uint32_t* __restrict__ item_band, const uint64_t* __restrict__ item0, const uint64_t* __restrict__ n_items,
    CamPack cp, int band_tiles, uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t s_d[];   // band tiles + 1
  __shared__ uint32_t s_off[64];
  const int lane = threadIdx.x;
  const uint64_t items = *n_items;
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
  __syncthreads();
  const uint32_t k = item_band[item];
  const Band B = band_of(cp, k);
  const int nt = B.n;
  for (int i = lane; i <= nt; i += 64) s_d[i] = 0u;
  __syncthreads();
  const uint64_t p0 = brange[2 * (uint64_t)k] + (item - item0[k]) * kBlockPairs;
  const uint64_t pe = brange[2 * (uint64_t)k + 1];
  const uint64_t p1 = p0 + kBlockPairs < pe ? p0 + kBlockPairs : pe;
  for (uint64_t i = p0 + lane; i < p1; i += 64) {
    const uint4 d = desc[pval[i]];
    const int tx0 = (int)(d.y & 0xffffu), w = (int)(d.y >> 16);
    const int ty0 = (int)(d.z & 0xffffu), ty1 = (int)(d.z >> 16);
    const int ya = ty0 > B.r0 ? ty0 : B.r0, yb = ty1 < B.r1 - 1 ? ty1 : B.r1 - 1;
    for (int y = ya; y <= yb; ++y) {
      const int a = (y - B.r0) * B.tx + tx0;
      atomicAdd(&s_d[a], 1u);
      atomicSub(&s_d[a + w], 1u);
    }
  }
  __syncthreads();
  const int chunk = (nt + 63) / 64;
  const int c0 = lane * chunk, c1 = c0 + chunk < nt ? c0 + chunk : nt;
  uint32_t run = 0;
  for (int i = c0; i < c1; ++i) {
    run += s_d[i];
    s_d[i] = run;
  }
  uint32_t tot;
  s_off[lane] = wave_excl_scan_u32(run, lane, &tot);
  __syncthreads();
  uint32_t* dst = counts + item * (uint64_t)band_tiles;
  for (int i = lane; i < nt; i += 64) dst[i] = s_d[i] + s_off[i / chunk];
  }
}


// Tile scans over the items of a band, in groups of kItemGroup items: one
// wavefront per (band, 64-tile chunk, group) so that thousands of
// wavefronts share the work.  Pass 1 stores each group's per-tile sum (in
// the group's first item row of `gsum`) and adds it to the tile total.
__global__ __launch_bounds__(64) void place_group_sums_kernel(
    const uint32_t* __restrict__ counts, const uint32_t* __restrict__ nitems, const uint64_t* __restrict__ item0,
    CamPack cp, int band_tiles, int64_t n_bands, int chunks, int groups, uint32_t* __restrict__ gsum,
    uint32_t* __restrict__ totals) {
  const int64_t w = blockIdx.x;
  const int64_t k = w / ((int64_t)chunks * groups);
  const int rem = (int)(w - k * (int64_t)chunks * groups);
  const int chunk = rem / groups, g = rem % groups;
  if (k >= n_bands) return;
  const Band B = band_of(cp, k);
  const int t = chunk * 64 + (int)threadIdx.x;
  const uint32_t ni = nitems[k];
  const uint32_t i0 = (uint32_t)g * kItemGroup;
  if (t >= B.n || i0 >= ni) return;
  const uint32_t i1 = i0 + kItemGroup < ni ? i0 + kItemGroup : ni;
  const uint32_t* c = counts + item0[k] * (uint64_t)band_tiles + t;
  uint32_t v = 0;
#pragma unroll 8
  for (uint32_t i = i0; i < i1; ++i) v += c[(uint64_t)i * band_tiles];
  gsum[(item0[k] + i0) * (uint64_t)band_tiles + t] = v;
  atomicAdd(&totals[B.lo + t], v);
}

// Pass 2: counts[item][t] <- position of the item's first entry of tile t
// (tile start + the groups before + the items before in the group); the
// ranges ([0, 0) for an empty tile, and for every tile when the entries
// overflow the capacity).
__global__ __launch_bounds__(64) void place_offsets_kernel(
    uint32_t* __restrict__ counts, const uint32_t* __restrict__ gsum, const uint32_t* __restrict__ nitems,
    const uint64_t* __restrict__ item0, const uint32_t* __restrict__ totals, const uint64_t* __restrict__ starts,
    const uint64_t* __restrict__ n_dup, int64_t capacity, CamPack cp, int band_tiles, int64_t n_bands, int chunks,
    int groups, uint32_t* __restrict__ ranges) {
  const int64_t w = blockIdx.x;
  const int64_t k = w / ((int64_t)chunks * groups);
  const int rem = (int)(w - k * (int64_t)chunks * groups);
  const int chunk = rem / groups, g = rem % groups;
  if (k >= n_bands) return;
  const Band B = band_of(cp, k);
  const int t = chunk * 64 + (int)threadIdx.x;
  if (t >= B.n) return;
  const bool over = *n_dup > (uint64_t)capacity;
  const uint64_t tg = B.lo + (uint64_t)t;
  // every load before the first store: the vector memory counter orders
  // loads and stores, so a load behind a store would wait for it (and the
  // group's counts read and overwritten one by one would wait item by item)
  const uint32_t a = (uint32_t)starts[tg];
  const uint32_t tot = g == 0 ? totals[tg] : 0u;
  const uint32_t ni = nitems[k];
  const uint64_t row0 = item0[k];
  const uint32_t i0 = (uint32_t)g * kItemGroup;
  const bool mine = !over && i0 < ni;
  const uint32_t i1 = i0 + kItemGroup < ni ? i0 + kItemGroup : ni;
  uint32_t* c = counts + row0 * (uint64_t)band_tiles + t;
  uint32_t run = a;
  uint32_t v[kItemGroup];
  if (mine) {
    for (uint32_t gi = 0; gi < i0; gi += kItemGroup) run += gsum[(row0 + gi) * (uint64_t)band_tiles + t];
#pragma unroll
    for (int j = 0; j < kItemGroup; ++j) v[j] = i0 + j < i1 ? c[(uint64_t)(i0 + j) * band_tiles] : 0u;
  }
  if (g == 0) {
    ranges[2 * tg] = (tot && !over) ? a : 0u;
    ranges[2 * tg + 1] = (tot && !over) ? a + tot : 0u;
  }
  if (!mine) return;
#pragma unroll
  for (int j = 0; j < kItemGroup; ++j) {
    if (i0 + j < i1) c[(uint64_t)(i0 + j) * band_tiles] = run;
    run += v[j];
  }
}

// The entries of one item, staged in LDS.  Each wavefront takes
// kEmitPerWave consecutive pairs (records in depth order).  Pass 1 counts
// per wavefront how many of its records cover each tile of the band; a scan
// across the wavefronts turns the counts into per-wavefront cursors, and a
// scan over the tiles lays the item's runs (one per tile, in tile order)
// out in the staging area.  Pass 2 walks every wavefront's records one
// after another (covered tiles across the lanes) and takes each entry's
// slot with an LDS fetch-and-add, so a tile's slots follow record order.
// Each run is then copied to its place in the tile's list in one contiguous
// burst.  An item with more entries than the staging area holds writes its
// entries straight to their final positions instead.
//
// Bands of up to kEmitWideTiles tiles keep a 32-bit cursor per (wavefront,
// tile), counted with a difference array (two LDS increments per record
// row, lanes = records) and holding absolute slots.  Wider bands (one tile
// row of a very wide image) pack two wavefronts' 16-bit cursors, relative
// to the run, per word, and count entry by entry.
constexpr int kEmitWaves = 8;
constexpr int kEmitThreads = kEmitWaves * 64;
constexpr int kEmitPerWave = kBlockPairs / kEmitWaves;
static_assert(kEmitPerWave == 64, "one pair per lane in the decode");
static_assert(kBlockPairs < 65536, "16-bit cursors");
constexpr int kEmitWideTiles = 512;
constexpr size_t kEmitLdsBytes = 32768 - 512;  // dynamic part; the static s_wsum and s_spare sit beside it

// LDS words of the cursor area per tile, and the fixed part in bytes.
inline bool emit_packed(int band_tiles) { return band_tiles > kEmitWideTiles; }
inline size_t emit_fixed_lds(int band_tiles) {
  const size_t cur = emit_packed(band_tiles) ? (size_t)(kEmitWaves / 2) * band_tiles
                                             : (size_t)kEmitWaves * (band_tiles + 1);
  return (cur + 2 * (size_t)band_tiles + 1) * sizeof(uint32_t);
}

// Entry e of a record's band part -> its local tile (rows of width W
// starting at local tile `base`, band row pitch tx).  n <= 2 W (at most two
// rows, the common case) needs no division.
__device__ __forceinline__ int entry_tile(int e, int W, int n, float inv_w, int base, int tx) {
  if (n <= 2 * W) return base + (e >= W ? tx - W : 0) + e;
  int row = (int)((float)e * inv_w);
  int col = e - row * W;
  if (col < 0) { --row; col += W; }
  if (col >= W) { ++row; col -= W; }
  return base + row * tx + col;
}

template <bool PACKED>
__global__ __launch_bounds__(kEmitThreads) void place_emit_kernel(
    const uint4* __restrict__ desc, const uint32_t* __restrict__ pval, const uint32_t* __restrict__ brange,
    const uint32_t* __restrict__ item_band, const uint64_t* __restrict__ item0, const uint64_t* __restrict__ n_items,
    CamPack cp, int band_tiles, int stage_cap, const uint32_t* __restrict__ offsets,
    const uint64_t* __restrict__ n_dup, int64_t capacity, int32_t* __restrict__ overflow,
    uint32_t* __restrict__ vals) {
  extern __shared__ uint32_t lds[];
  // cursor area: PACKED [kEmitWaves / 2][band_tiles] (2 x 16 bits), else
  // [kEmitWaves][band_tiles + 1]
  constexpr int kCurRows = PACKED ? kEmitWaves / 2 : kEmitWaves;
  const int pitch = PACKED ? band_tiles : band_tiles + 1;
  uint32_t* s_cur = lds;
  uint32_t* s_start = s_cur + kCurRows * pitch;     // [band_tiles + 1] run start in the staging area
  uint32_t* s_off = s_start + band_tiles + 1;       // [band_tiles] run start in the tile's list
  uint32_t* s_stage = s_off + band_tiles;           // [stage_cap]
  __shared__ uint32_t s_wsum[kEmitWaves];
  __shared__ uint32_t s_spare[64];   // target of the walk's idle lanes
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool over = *n_dup > (uint64_t)capacity;
  if (blockIdx.x == 0 && tid == 0) *overflow = over ? 1 : 0;
  if (over) return;
  const uint64_t items = *n_items;
  for (uint64_t item = blockIdx.x; item < items; item += gridDim.x) {
  __syncthreads();   // the previous item's copy-out is done with the LDS
  const uint32_t k = item_band[item];
  const Band B = band_of(cp, k);
  const int nt = B.n;
  for (int i = tid; i < kCurRows * pitch; i += kEmitThreads) s_cur[i] = 0u;
  const uint32_t* src = offsets + item * (uint64_t)band_tiles;
  for (int i = tid; i < nt; i += kEmitThreads) s_off[i] = src[i];
  // this wavefront's pairs, one per lane: record, width, first local tile,
  // rows in the band, entries in the band
  const uint64_t p0 = brange[2 * (uint64_t)k] + (item - item0[k]) * kBlockPairs;
  const uint64_t pe = brange[2 * (uint64_t)k + 1];
  const uint64_t w0 = p0 + (uint64_t)wv * kEmitPerWave;
  const uint64_t w1 = w0 + kEmitPerWave < pe ? w0 + kEmitPerWave : pe;
  const int cnt = w1 > w0 ? (int)(w1 - w0) : 0;
  uint32_t dR = 0, dW = 1;
  int dbase = 0, dn = 0, drows = 0;
  if (lane < cnt) {
    const uint4 d = desc[pval[w0 + lane]];
    const int tx0 = (int)(d.y & 0xffffu), ty0 = (int)(d.z & 0xffffu), ty1 = (int)(d.z >> 16);
    const int ya = ty0 > B.r0 ? ty0 : B.r0, yb = ty1 < B.r1 - 1 ? ty1 : B.r1 - 1;
    dR = d.x;
    dW = d.y >> 16;
    dbase = (ya - B.r0) * B.tx + tx0;
    drows = yb - ya + 1;
    dn = (int)dW * drows;
  }
  uint32_t* cur = s_cur + (PACKED ? (wv >> 1) : wv) * pitch;
  const int half = PACKED ? (wv & 1) * 16 : 0;
  const uint32_t inc = 1u << half;
  __syncthreads();
  // pass 1: this wavefront's count per tile
  if constexpr (PACKED) {
    for (int l = 0; l < cnt; ++l) {
      const int W = __builtin_amdgcn_readlane((int)dW, l);
      const int base = __builtin_amdgcn_readlane(dbase, l);
      const int n = __builtin_amdgcn_readlane(dn, l);
      const float inv_w = __builtin_amdgcn_rcpf((float)W);
      for (int q = 0; q < n; q += 64) {
        const int e = q + lane;
        const int t = entry_tile(e, W, n, inv_w, base, B.tx);
        if (e < n) atomicAdd(&cur[t], inc);
      }
    }
  } else {
    // difference array over the band's linear tile index: +1 at a row's
    // first tile, -1 after its last (modular arithmetic; the prefix sums
    // are the counts)
    for (int r = 0; r < drows; ++r) {
      const int a = dbase + r * B.tx;
      atomicAdd(&cur[a], 1u);
      atomicSub(&cur[a + (int)dW], 1u);
    }
  }
  __syncthreads();
  if constexpr (!PACKED) {
    // each wavefront's prefix sum over its own difference array
    const int chunk = (nt + 63) / 64;
    const int c0 = lane * chunk, c1 = c0 + chunk < nt ? c0 + chunk : nt;
    uint32_t run = 0;
    for (int i = c0; i < c1; ++i) {
      run += cur[i];
      cur[i] = run;
    }
    uint32_t tot;
    const uint32_t ex = wave_excl_scan_u32(run, lane, &tot);
    for (int i = c0; i < c1; ++i) cur[i] += ex;
    __syncthreads();
  }
  // per tile: counts -> offsets across the wavefronts (relative to the
  // run), the run length; then the runs laid out in tile order
  const int per = (nt + kEmitThreads - 1) / kEmitThreads;
  const int t0 = tid * per, t1 = t0 + per < nt ? t0 + per : nt;
  uint32_t mine = 0;
  for (int t = t0; t < t1; ++t) {
    uint32_t run = 0;
    if constexpr (PACKED) {
#pragma unroll
      for (int p = 0; p < kEmitWaves / 2; ++p) {
        const uint32_t c = s_cur[p * pitch + t];
        const uint32_t lo = run, hi = run + (c & 0xffffu);
        s_cur[p * pitch + t] = lo | (hi << 16);
        run = hi + (c >> 16);
      }
    } else {
#pragma unroll
      for (int w = 0; w < kEmitWaves; ++w) {
        const uint32_t c = s_cur[w * pitch + t];
        s_cur[w * pitch + t] = run;
        run += c;
      }
    }
    s_start[t] = run;
    mine += run;
  }
  uint32_t wtot;
  const uint32_t wex = wave_excl_scan_u32(mine, lane, &wtot);
  if (lane == 0) s_wsum[wv] = wtot;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < kEmitWaves; ++w) {
    const uint32_t x = s_wsum[w];
    before += w < wv ? x : 0u;
    total += x;
  }
  const bool staged = total <= (uint32_t)stage_cap;
  uint32_t at = before + wex;
  for (int t = t0; t < t1; ++t) {
    const uint32_t len = s_start[t];
    s_start[t] = at;
    if constexpr (!PACKED) {
      // absolute slots: in the staging area, or in the tile's list
      const uint32_t base = staged ? at : s_off[t];
#pragma unroll
      for (int w = 0; w < kEmitWaves; ++w) s_cur[w * pitch + t] += base;
    }
    at += len;
  }
  if (tid == 0) s_start[nt] = total;
  __syncthreads();
  // pass 2: slots in record order per tile
  uint32_t* dst = staged ? s_stage : vals;
  const uint32_t* run_base = staged ? s_start : s_off;
  auto walk_one = [&](int l) {
    const int n = __builtin_amdgcn_readlane(dn, l);
    const uint32_t R = (uint32_t)__builtin_amdgcn_readlane((int)dR, l);
    const int W = __builtin_amdgcn_readlane((int)dW, l);
    const int base = __builtin_amdgcn_readlane(dbase, l);
    const float inv_w = __builtin_amdgcn_rcpf((float)W);
    for (int q = 0; q < n; q += 64) {
      const int e = q + lane;
      const int t = entry_tile(e, W, n, inv_w, base, B.tx);
      if (e < n) {
        if constexpr (PACKED) {
          const uint32_t rel = (atomicAdd(&cur[t], inc) >> half) & 0xffffu;
          dst[run_base[t] + rel] = R;
        } else {
          dst[atomicAdd(&cur[t], 1u)] = R;
        }
      }
    }
  };
  int l = 0;
  if constexpr (!PACKED) {
    // four records at a time while each has at most 64 entries in the
    // band: their four fetch-and-adds are in flight together instead of one
    // round trip per record.  A tile that several of them cover still gets
    // its slots in record order: a wavefront's LDS operations complete in
    // the order it issues them.
    constexpr int G = 4;
    for (; l + G <= cnt; l += G) {
      int n[G], t[G];
      uint32_t R[G], slot[G];
      int nmax = 0;
#pragma unroll
      for (int k = 0; k < G; ++k) {
        n[k] = __builtin_amdgcn_readlane(dn, l + k);
        nmax = n[k] > nmax ? n[k] : nmax;
      }
      if (nmax > 64) {
#pragma unroll
        for (int k = 0; k < G; ++k) walk_one(l + k);
        continue;
      }
#pragma unroll
      for (int k = 0; k < G; ++k) {
        R[k] = (uint32_t)__builtin_amdgcn_readlane((int)dR, l + k);
        const int W = __builtin_amdgcn_readlane((int)dW, l + k);
        const int base = __builtin_amdgcn_readlane(dbase, l + k);
        t[k] = entry_tile(lane, W, n[k], __builtin_amdgcn_rcpf((float)W), base, B.tx);
      }
      // every lane issues each fetch-and-add (lanes past a record's entries
      // on a word of their own), so no branch separates the four and they
      // are in flight together
#pragma unroll
      for (int k = 0; k < G; ++k) slot[k] = atomicAdd(lane < n[k] ? &cur[t[k]] : &s_spare[lane], 1u);
#pragma unroll
      for (int k = 0; k < G; ++k)
        if (lane < n[k]) dst[slot[k]] = R[k];
    }
  }
  for (; l < cnt; ++l) walk_one(l);
  if (!staged) continue;
  __syncthreads();
  // copy out, one tile run per wavefront step: contiguous in the staging
  // area and in the tile's list
  for (int t = wv; t < nt; t += kEmitWaves) {
    const uint32_t a = s_start[t], e = s_start[t + 1];
    const uint32_t o = s_off[t];
    for (uint32_t i = a + lane; i < e; i += 64) vals[o + (i - a)] = s_stage[i];
  }
  }
}

// ---------------------------------------------------------------------------
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct SortWs {
  // placement path
  uint32_t* rkeys[2];
  uint32_t* rids[2];
  uint4* desc;         // [n_rec] tile rectangles in depth order
  uint32_t* nbands;    // [n_rec]
  uint64_t* poff;      // [n_rec] first pair of each slot
  uint32_t* pkey[2];   // [pairs_max] band of each (record, band) pair
  uint32_t* pval[2];   // [pairs_max] its slot
  uint32_t* brange;    // [n_bands][2]
  uint32_t* nitems;    // [n_bands]
  uint64_t* item0;     // [n_bands]
  uint32_t* item_band; // [items_max]
  uint32_t* counts;    // [items_max][band_tiles], then offsets
  uint32_t* gsum;      // [items_max][band_tiles]: per item group, at its first item
  uint32_t* totals;    // [n_tiles]
  uint64_t* starts;    // [n_tiles]
  uint64_t* scalars;   // n_pairs, n_items, tile total
  void* scan_ws;
  // full-key path
  uint64_t* alt_keys64;
  uint32_t* alt_vals;
  uint32_t* chunk_start;
  // both paths
  uint32_t* okeys[2];  // tile order sort
  uint32_t* oalt;
  uint32_t* hist;      // [kHistCopies][2][kMaxPasses][256]: record passes, entry (or pair) passes
  uint32_t* bases;     // [2][kMaxPasses][256] scanned
  uint32_t* tickets;   // [2][kMaxPasses]
  uint64_t* lookback[2];
  int64_t parts;
  PlaceGeom geom;
  size_t bytes;
};

SortWs carve(void* ws, int64_t n_rec, int64_t capacity, const CamPack& cp, bool full_keys) {
  const int64_t n_tiles = (int64_t)cp.tiles_total;
  SortWs w{};
  w.geom = place_geom(n_rec, capacity, cp);
  const PlaceGeom& g = w.geom;
  int64_t small = n_rec > n_tiles ? n_rec : n_tiles;
  if (!full_keys) small = small > g.pairs_max ? small : g.pairs_max;
  const int64_t pe = full_keys ? (capacity + kPartMinEntries - 1) / kPartMinEntries : 0;
  const int64_t ps = (small + kPartMinSmall - 1) / kPartMinSmall;
  const int64_t parts = pe > ps ? pe : ps;
  w.parts = parts > 0 ? parts : 1;
  const size_t nr = (size_t)(n_rec > 0 ? n_rec : 1), cap = (size_t)(capacity > 0 ? capacity : 1);
  const size_t nt = (size_t)(n_tiles > 0 ? n_tiles : 1);
  const size_t nbd = (size_t)g.n_bands, np = (size_t)g.pairs_max, ni = (size_t)g.items_max;
  char* p = (char*)ws;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void* q = p ? (void*)(p + off) : nullptr;
    off += align256(bytes);
    return q;
  };
  if (full_keys) {
    w.alt_keys64 = (uint64_t*)take(cap * 8);
    w.alt_vals = (uint32_t*)take(cap * 4);
    w.chunk_start = (uint32_t*)take((cap + kChunk - 1) / kChunk * 4 + 4);
  } else {
    for (int b = 0; b < 2; ++b) w.rkeys[b] = (uint32_t*)take(nr * 4);
    for (int b = 0; b < 2; ++b) w.rids[b] = (uint32_t*)take(nr * 4);
    w.desc = (uint4*)take(nr * 16);
    w.nbands = (uint32_t*)take(nr * 4);
    w.poff = (uint64_t*)take(nr * 8);
    for (int b = 0; b < 2; ++b) w.pkey[b] = (uint32_t*)take(np * 4);
    for (int b = 0; b < 2; ++b) w.pval[b] = (uint32_t*)take(np * 4);
    w.brange = (uint32_t*)take(nbd * 8);
    w.nitems = (uint32_t*)take(nbd * 4);
    w.item0 = (uint64_t*)take(nbd * 8);
    w.item_band = (uint32_t*)take(ni * 4);
    w.counts = (uint32_t*)take(ni * (size_t)g.band_tiles * 4);
    w.gsum = (uint32_t*)take(ni * (size_t)g.band_tiles * 4);
    w.totals = (uint32_t*)take(nt * 4);
    w.starts = (uint64_t*)take(nt * 8);
    w.scalars = (uint64_t*)take(4 * 8);
    size_t sw = scan_workspace_bytes((int64_t)nr);
    const size_t s2 = scan_workspace_bytes((int64_t)nt), s3 = scan_workspace_bytes((int64_t)nbd);
    sw = sw > s2 ? sw : s2;
    sw = sw > s3 ? sw : s3;
    w.scan_ws = take(sw);
  }
  for (int b = 0; b < 2; ++b) w.okeys[b] = (uint32_t*)take(nt * 4);
  w.oalt = (uint32_t*)take(nt * 4);
  w.hist = (uint32_t*)take((size_t)kHistCopies * kHistWords * 4);
  w.bases = (uint32_t*)take((size_t)kHistWords * 4);
  w.tickets = (uint32_t*)take((size_t)2 * kMaxPasses * 4);
  for (int b = 0; b < 2; ++b) w.lookback[b] = (uint64_t*)take((size_t)w.parts * kRadix * 8);
  w.bytes = off;
  return w;
}

unsigned grid_for(int64_t items, int64_t per_block, int64_t cap) {
  int64_t g = (items + per_block - 1) / per_block;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

// The passes of one sort phase (same key count bound `cap`, so every pass has
// the same number of partitions).  A pass reads look-back buffer lb and
// clears the other one over its partitions for the next pass; the first
// buffer is cleared here over the phase's partition bound, so no state from
// an earlier phase (with a different partition count) survives.
template <typename K, int ITEMS>
void onesweep_passes(K** kb, uint32_t** vb, const uint64_t* n_dev, int64_t cap, int first_shift,
                     int passes, const uint32_t* bases, SortWs& w, uint32_t* tickets, int& lb,
                     hipStream_t s) {
  constexpr int PART = kBlock * ITEMS;
  const int64_t parts = (cap + PART - 1) / PART > 0 ? (cap + PART - 1) / PART : 1;
  const unsigned grid = (unsigned)(parts < kSweepGrid ? parts : kSweepGrid);
  if (passes <= 0) return;
  // look-back flags: sort_init_kernel cleared those of the call's first
  // pass, each pass clears the next one's
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((onesweep_kernel<K, ITEMS>), dim3(grid), dim3(kBlock), 0, s, kb[p & 1], vb[p & 1],
                       kb[(p + 1) & 1], vb[(p + 1) & 1], n_dev, cap, first_shift + 8 * p,
                       bases + p * kRadix, w.lookback[lb & 1], w.lookback[(lb + 1) & 1], w.parts * kRadix,
                       tickets + p);
    ++lb;
  }
}

}  // namespace

int tile_bits(uint32_t tiles_total) {
  int tb = 0;
  while ((1ull << tb) < tiles_total) ++tb;
  return tb;
}

size_t sort_workspace_bytes(int64_t n_rec, int64_t capacity, const CamPack& cp, bool full_keys) {
  return carve(nullptr, n_rec, capacity, cp, full_keys).bytes;
}

hipError_t launch_bin_sort(const Record* rec, const uint32_t* tiles, const uint64_t* offsets,
                           const uint64_t* n_dup, int64_t n_rec, int64_t n_per_cam,
                           const CamPack& cp, uint64_t* keys, uint32_t* vals, int64_t capacity,
                           uint32_t* ranges, uint32_t* tile_order, int32_t* overflow, void* ws,
                           bool full_keys, hipStream_t s) {
  SortWs w = carve(ws, n_rec, capacity, cp, full_keys);
  const int tb = tile_bits(cp.tiles_total);
  uint32_t* hist_rec = w.hist;                       // replica 0; replicas follow
  uint32_t* hist_ent = w.hist + kMaxPasses * kRadix;
  uint32_t* base_rec = w.bases;
  uint32_t* base_ent = w.bases + kMaxPasses * kRadix;
  int lb = 0;  // look-back buffer in use
  const int64_t n_brange = full_keys ? 0 : 2 * (int64_t)w.geom.n_bands;
  const int64_t n_totals = full_keys ? 0 : (int64_t)cp.tiles_total;
  int64_t n_init = kHistCopies * kHistWords > n_totals ? kHistCopies * kHistWords : n_totals;
  n_init = n_init > w.parts * kRadix ? n_init : w.parts * kRadix;
  hipLaunchKernelGGL(sort_init_kernel, dim3(grid_for(n_init, kBlock, 4096)), dim3(kBlock), 0, s, w.hist,
                     w.tickets, w.lookback[0], w.parts * kRadix, w.brange, n_brange, w.totals, n_totals);
  const unsigned dup_grid = grid_for((capacity + kChunk - 1) / kChunk, kWaves, 1 << 30);

  if (full_keys) {
    const int passes = (32 + tb + 7) / 8;
    uint64_t* kb[2];
    uint32_t* vb[2];
    if (passes % 2 == 0) {
      kb[0] = keys; vb[0] = vals; kb[1] = w.alt_keys64; vb[1] = w.alt_vals;
    } else {
      kb[0] = w.alt_keys64; vb[0] = w.alt_vals; kb[1] = keys; vb[1] = vals;
    }
    hipLaunchKernelGGL(depth_hist_weighted_kernel, dim3(grid_for(n_rec, kBlock, 2048)), dim3(kBlock), 0, s,
                       rec, tiles, n_rec, hist_ent);
    if (n_rec > 0)
      hipLaunchKernelGGL(chunk_start_kernel, dim3(grid_for(n_rec, kBlock, 1ll << 31)), dim3(kBlock), 0, s,
                         nullptr, tiles, offsets, n_rec, (uint64_t)((capacity + kChunk - 1) / kChunk),
                         w.chunk_start);
    hipLaunchKernelGGL(duplicate_kernel<true>, dim3(dup_grid), dim3(kBlock), 0, s, rec, nullptr, tiles,
                       offsets, (const uint32_t*)w.chunk_start, n_dup, n_rec, n_per_cam, cp, (void*)kb[0],
                       vb[0], capacity, overflow, hist_ent + 4 * kRadix, 32, passes - 4);
    hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(kHistScanThreads), 0, s, hist_ent, base_ent, passes);
    onesweep_passes<uint64_t, SweepItems<uint64_t>::value>(kb, vb, n_dup, capacity, 0, passes, base_ent, w,
                                                           w.tickets + kMaxPasses, lb, s);
    const int64_t nr = 2 * (int64_t)cp.tiles_total;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(nr, kBlock, 4096)), dim3(kBlock), 0, s, ranges, nr, 0u);
    if (capacity > 0)
      hipLaunchKernelGGL(ranges_kernel<uint64_t>, dim3(grid_for(capacity, kBlock, 1ll << 31)), dim3(kBlock),
                         0, s, keys, 32, n_dup, capacity, ranges);
  } else {
    // 1. records in (depth, id) order
    // the compact rectangles live in the pair-offset buffer, which is only
    // written after their last reader (place_desc_kernel)
    static_assert(sizeof(uint2) == sizeof(uint64_t), "one rectangle per pair offset");
    uint2* rects = reinterpret_cast<uint2*>(w.poff);
    hipLaunchKernelGGL(depth_keys_kernel, dim3(grid_for(n_rec, kBlock, 2048)), dim3(kBlock), 0, s, rec,
                       tiles, n_rec, w.rkeys[0], w.rids[0], hist_rec, rects, cp.tile_shift);
    hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(kHistScanThreads), 0, s, hist_rec, base_rec, 4);
    if (n_rec > 0)
      onesweep_passes<uint32_t, kSmallItems>(w.rkeys, w.rids, nullptr, n_rec, 0, 4, base_rec, w, w.tickets,
                                             lb, s);
    const uint32_t* order = w.rids[0];  // four passes: back in buffer 0
    const int64_t nt = (int64_t)cp.tiles_total;
    const PlaceGeom& g = w.geom;
    uint64_t* n_pairs = w.scalars;
    uint64_t* n_items = w.scalars + 1;
    // 2. tile rectangles in depth order, (band, slot) pairs sorted by band
    //    (stable: slots stay in depth order inside a band)
    hipLaunchKernelGGL(place_desc_kernel, dim3(grid_for(n_rec, kBlock, 1ll << 31)), dim3(kBlock), 0, s,
                       (const uint2*)rects, order, n_rec, n_per_cam, cp, w.desc, w.nbands);
    hipError_t e = launch_scan(w.nbands, n_rec, w.poff, n_pairs, w.scan_ws, s);
    if (e != hipSuccess) return e;
    const int bpasses = (g.band_bits + 7) / 8;
    hipLaunchKernelGGL(place_pairs_kernel, dim3(grid_for(n_rec, kBlock, 2048)), dim3(kBlock), 0, s,
                       (const uint4*)w.desc, (const uint32_t*)w.nbands, (const uint64_t*)w.poff, n_rec,
                       g.pairs_max, cp, g.n_bands, w.pkey[0], w.pval[0], hist_ent, bpasses);
    if (bpasses > 0) {
      hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(kHistScanThreads), 0, s, hist_ent, base_ent, bpasses);
      onesweep_passes<uint32_t, kSmallItems>(w.pkey, w.pval, n_pairs, g.pairs_max, 0, bpasses, base_ent, w,
                                             w.tickets + kMaxPasses, lb, s);
    }
    const uint32_t* pkey = w.pkey[bpasses & 1];
    const uint32_t* pval = w.pval[bpasses & 1];
    hipLaunchKernelGGL(place_band_ranges_kernel, dim3(grid_for(g.pairs_max, kBlock, 8192)), dim3(kBlock), 0, s,
                       pkey, (const uint64_t*)n_pairs, g.pairs_max, w.brange);
    hipLaunchKernelGGL(place_band_items_kernel, dim3(grid_for(g.n_bands, kBlock, 1ll << 31)), dim3(kBlock), 0, s,
                       (const uint32_t*)w.brange, g.n_bands, w.nitems);
    e = launch_scan(w.nitems, g.n_bands, w.item0, n_items, w.scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(place_item_bands_kernel, dim3(grid_for(g.items_max, kBlock, 1024)), dim3(kBlock), 0, s,
                       (const uint32_t*)w.nitems, (const uint64_t*)w.item0, (const uint64_t*)n_items, g.n_bands,
                       w.item_band);
    // 3. counts[item][tile], tile totals, their scan, per-item offsets, ranges
    const size_t lds = (size_t)(g.band_tiles + 1) * sizeof(uint32_t);
    const unsigned items = (unsigned)(g.items_max < kItemGrid ? g.items_max : kItemGrid);
    hipLaunchKernelGGL(place_count_kernel, dim3(items), dim3(64), lds, s, (const uint4*)w.desc, pval,
                       (const uint32_t*)w.brange, (const uint32_t*)w.item_band, (const uint64_t*)w.item0,
                       (const uint64_t*)n_items, cp, g.band_tiles, w.counts);
    // tile totals by groups of items (a band holds at most n_per_cam pairs)
    const int chunks = (g.band_tiles + 63) / 64;
    const int64_t items_band = (n_per_cam + kBlockPairs - 1) / kBlockPairs;
    const int groups = (int)((items_band + kItemGroup - 1) / kItemGroup > 0 ? (items_band + kItemGroup - 1) / kItemGroup : 1);
    const unsigned scan_grid = (unsigned)(g.n_bands * chunks * groups);
    hipLaunchKernelGGL(place_group_sums_kernel, dim3(scan_grid), dim3(64), 0, s, (const uint32_t*)w.counts,
                       (const uint32_t*)w.nitems, (const uint64_t*)w.item0, cp, g.band_tiles, g.n_bands, chunks,
                       groups, w.gsum, w.totals);
    e = launch_scan(w.totals, nt, w.starts, w.scalars + 2, w.scan_ws, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(place_offsets_kernel, dim3(scan_grid), dim3(64), 0, s, w.counts, (const uint32_t*)w.gsum,
                       (const uint32_t*)w.nitems, (const uint64_t*)w.item0, (const uint32_t*)w.totals,
                       (const uint64_t*)w.starts, n_dup, capacity, cp, g.band_tiles, g.n_bands, chunks, groups,
                       ranges);
    // 4. the entries
    const size_t emit_fixed = emit_fixed_lds(g.band_tiles);
    const int stage_cap = emit_fixed < kEmitLdsBytes ? (int)((kEmitLdsBytes - emit_fixed) / sizeof(uint32_t)) : 0;
    const size_t emit_lds = emit_fixed + (size_t)stage_cap * sizeof(uint32_t);
    if (emit_packed(g.band_tiles))
      hipLaunchKernelGGL(place_emit_kernel<true>, dim3(items), dim3(kEmitThreads), emit_lds, s,
                         (const uint4*)w.desc, pval, (const uint32_t*)w.brange, (const uint32_t*)w.item_band,
                         (const uint64_t*)w.item0, (const uint64_t*)n_items, cp, g.band_tiles, stage_cap,
                         (const uint32_t*)w.counts, n_dup, capacity, overflow, vals);
    else
      hipLaunchKernelGGL(place_emit_kernel<false>, dim3(items), dim3(kEmitThreads), emit_lds, s,
                         (const uint4*)w.desc, pval, (const uint32_t*)w.brange, (const uint32_t*)w.item_band,
                         (const uint64_t*)w.item0, (const uint64_t*)n_items, cp, g.band_tiles, stage_cap,
                         (const uint32_t*)w.counts, n_dup, capacity, overflow, vals);
    if (keys)
      hipLaunchKernelGGL(keys_from_ranges_kernel, dim3(nt > 0 ? (unsigned)nt : 1u), dim3(64), 0, s,
                         (const uint32_t*)ranges, (const uint32_t*)vals, rec, nt, keys);
  }
  // 6. tiles by decreasing list length, for the persistent raster
  if (tile_order) {
    const int64_t nt = (int64_t)cp.tiles_total;
    uint32_t* ob[2] = {w.okeys[0], w.okeys[1]};
    uint32_t* ov[2] = {w.oalt, tile_order};  // one pass: the order lands in tile_order
    hipLaunchKernelGGL(order_keys_kernel, dim3(grid_for(nt, kBlock, 1024)), dim3(kBlock), 0, s, ranges, nt,
                       ob[0], ov[0], hist_rec + 4 * kRadix);
    hipLaunchKernelGGL(hist_scan_kernel, dim3(1), dim3(kHistScanThreads), 0, s, hist_rec + 4 * kRadix,
                       base_rec + 4 * kRadix, 1);
    onesweep_passes<uint32_t, kSmallItems>(ob, ov, nullptr, nt, 0, 1, base_rec + 4 * kRadix, w, w.tickets + 4,
                                           lb, s);
  }
  return hipGetLastError();
}

}  // namespace hgs
