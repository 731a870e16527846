// Tile rasterizer: per-pixel front-to-back blending with the paired-half
// opacity of Eq. 10, and its back-to-front replay for gradients.
//
// Work decomposition (CDNA, wave64): a wavefront owns a 16x16 block of
// pixels (8x8 for 8-pixel tiles) and each lane owns 4 pixels of it (1 for
// 8-pixel tiles) -- pixel rows ly, ly+4, ly+8, ly+12 of column lx.  A 32-pixel
// tile is four such wavefronts walking the same list.  Every lane of a
// wavefront needs the same record at the same time, so the list is walked
// with wave-uniform indices: a round fetches `batch` entry ids with one
// vector load per lane, then each id is broadcast with v_readlane and its
// 64-byte record is loaded as uniform (scalar) data, whole, in one
// request.  No workgroup barriers: each wavefront stops as soon as all of
// its pixels are done.
//
// Backward: each lane replays its pixels back to front from the last blended
// entry, dividing the transmittance back out, and sums its pixels'
// gradients for the entry; the 12 sums are then reduced across the 64 lanes
// (DPP and lane swaps, reduce-scatter) and four lanes issue the float atomics,
// so there is one reduction and one set of atomics per (entry, 256 pixels).

#include "hgs_internal.h"

// Every fused multiply-add below is written out: with contraction left to the
// compiler, instantiations with different pixels-per-lane fused differently
// and images depended on the tile size in the last bit.
#pragma clang fp contract(off)

namespace hgs {

namespace {

constexpr float kTwoOverSqrtPi = 1.12837916709551257390f;

// erfc(x) for the half factor.  For z = |x| <= 3.9, log2 erfc(z) is smooth
// and is fitted by a degree-10 polynomial (least squares in the Chebyshev
// basis of [0, 3.9], coefficients rounded to float and checked in float
// Horner arithmetic: absolute error below 5e-8); beyond 3.9 the argument is
// clamped (erfc(3.9) = 3.5e-8).  erfc(-z) = 2 - erfc(z).  No reciprocal,
// one exp2, ten fma; branch-free, result in [0, 2].
__device__ __forceinline__ float erfc_fast(float x) {
  const float z = __builtin_amdgcn_fmed3f(fabsf(x), 0.0f, 3.9f);   // min(|x|, 3.9), one instruction
  float p = -1.3359800732359872e-06f;
  p = fmaf(p, z, 2.5692050257930532e-05f);
  p = fmaf(p, z, -0.00021396989177446812f);
  p = fmaf(p, z, 0.0009886942571029067f);
  p = fmaf(p, z, -0.0024599749594926834f);
  p = fmaf(p, z, 0.0002238718152511865f);
  p = fmaf(p, z, 0.027670344337821007f);
  p = fmaf(p, z, -0.1483006626367569f);
  p = fmaf(p, z, -0.9184418320655823f);
  p = fmaf(p, z, -1.6279075145721436f);
  p = fmaf(p, z, 6.547596242967302e-09f);
  const float e = __builtin_amdgcn_exp2f(p);
  return x >= 0.0f ? e : 2.0f - e;
}

constexpr float kLog2e = 1.44269504088896340736f;

// min(amax, HG) for HG >= 0 (alpha2 >= 0, alpha2 + d_o I lies between the two
// opacities, G >= 0): the median of (HG, 0, amax) is the same value, in one
// instruction instead of a canonicalising max and a min.
__device__ __forceinline__ float clamp_alpha(float hg, float amax) {
  return __builtin_amdgcn_fmed3f(hg, 0.0f, amax);
}

// Per-record values that do not depend on the lane (computed once per
// wavefront): a bound below which no pair of the record can reach alpha_min
// (see below) and the rect corner as floats.
struct RecordU {
  float hb;          // max(alpha2, alpha2 + 2 d_o) >= alpha2 + d_o I for I in [0, 2]
  float p2_min;      // log2(alpha_min) - log2(hb) less a margin of 2^-10
  float x0f, y0f;
  float y1p;         // y1 + 1/2: a pixel row py lies in the rect iff y0 < py + 1/2 < y1 + 1
  bool split;        // d_o != 0
};

// `log2_amin` = log2(alpha_min), once per kernel.
__device__ __forceinline__ RecordU record_uniform(const Record& r, int x0, int y0, int y1, float log2_amin) {
  RecordU u;
  u.hb = fmaxf(r.alpha2, fmaf(r.d_o, 2.0f, r.alpha2));
  u.p2_min = (log2_amin - __builtin_amdgcn_logf(u.hb)) - 0.0009765625f;
  u.x0f = (float)x0;
  u.y0f = (float)y0;
  u.y1p = (float)y1 + 1.0f;
  u.split = r.d_o != 0.0f;
  return u;
}

// Per-record values that a lane's pixels share (they lie in one column).
// fpx = px + 1/2 is the pixel centre; fpx - x0 is exact in float.
// p2 = log2(e) power is a quadratic in the row offset dy with per-column
// coefficients, p2 = p2a + p2b dy + p2c dy^2 (p2a = -log2(e)/2 qa dx^2,
// p2b = -log2(e) qb dx, p2c = -log2(e)/2 qc once per record), so a strip
// evaluates it in two multiply-adds.
struct Column {
  float dx, qadx, qbdx, kxdx;
  float p2a, p2b;
};

__device__ __forceinline__ Column column_of(const Record& r, const RecordU& u, float fpx) {
  Column c;
  c.dx = (fpx - u.x0f) - r.mx;
  c.qadx = r.qa * c.dx;
  c.qbdx = r.qb * c.dx;
  c.kxdx = r.kx * c.dx;
  c.p2a = r.qa * ((c.dx * c.dx) * (-0.5f * kLog2e));
  c.p2b = r.qb * (c.dx * -kLog2e);
  return c;
}

// One pixel against one record, in stages that the lanes of a wavefront
// skip together.  Every decision is a 64-bit lane mask (ballots of single
// comparisons, combined on the scalar unit), and per-lane updates select on
// a mask; forward and backward evaluate the same expressions, so they take
// identical decisions.
//   1. rect: pixel centre in the record's rect (column and row masks).
//   2. p2 = log2(e) power, power = -q / 2 of the dilated conic (so that
//      G = exp2(p2)); p2 <= 0 and p2 >= p2_min.  A pair below p2_min has
//      G * hb < alpha_min for the rounded G too (the 2^-10 margin covers the
//      exp2 and log2 rounding), so it cannot reach alpha_min: the skip is
//      exact.
//   3. G = exp2(p2); G * hb >= alpha_min (hb bounds alpha2 + d_o I since I
//      lies in [0, 2] and every rounding is monotone).
//   4. half factor I (Eq. 7-8), HG = (alpha2 + d_o I) G (Eq. 10),
//      alpha = min(alpha_max, HG) >= alpha_min.
__device__ __forceinline__ uint64_t lanes(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool in_mask(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

__device__ __forceinline__ float gauss_p2(const Column& c, float p2c, float dy) {
  return fmaf(fmaf(p2c, dy, c.p2b), dy, c.p2a);
}

// I = erfc(x), x = -(k . offset).  When every lane of mask m has |x| >= 3.9
// the polynomial is clamped for all of them, and I is erfc_fast(3.9) or
// 2 - erfc_fast(3.9) (`e39`, once per kernel): the same bits, no polynomial.
__device__ __forceinline__ float half_factor(const Record& r, const RecordU& u, const Column& c, float dy,
                                             uint64_t m, float e39) {
  if (!u.split) return 1.0f;
  const float x = -fmaf(r.ky, dy, c.kxdx);
  if ((lanes(fabsf(x) < 3.9f) & m) == 0ull) return x >= 0.0f ? e39 : 2.0f - e39;
  return erfc_fast(x);
}

// A wavefront's block is SUB x SUB pixels; lane l holds column l % SUB of
// rows l / SUB + j * ROWSTEP (j < PPL), so "strip" j is ROWSTEP full rows.
template <int T>
struct Geometry {
  static constexpr int SUB = (T == 8) ? 8 : 16;       // pixels per wavefront side
  static constexpr int PPL = SUB * SUB / 64;          // pixels per lane
  static constexpr int WAVES = (T / SUB) * (T / SUB); // wavefronts per tile
  static constexpr int ROWSTEP = 64 / SUB;            // rows between a lane's pixels

};

// The backward pass uses taller blocks at 32-pixel tiles: SUBX x SUBY pixels
// per wavefront (16 x 32, two wavefronts per tile, 8 pixels per lane), so
// that the per-entry work of a wavefront -- record setup, the 12-value
// reduction and the atomics -- is shared by twice the pixels.
template <int T>
struct BwdGeometry {
  static constexpr int SUBX = (T == 8) ? 8 : 16;
  static constexpr int SUBY = (T == 32) ? 32 : SUBX;
  static constexpr int PPL = SUBX * SUBY / 64;
  static constexpr int WAVES = (T / SUBX) * (T / SUBY);
  static constexpr int ROWSTEP = 64 / SUBX;
};

// Strip marks.  One byte per tile-list position and forward wavefront: bit
// j set if some pixel of the wavefront's strip j took that entry.  The
// backward pass replays exactly the blended pairs -- the same expressions
// give the same decisions, and a pixel's pairs at or before its last
// blended entry that pass the tests are the pairs it blended -- so it
// visits only marked entries, and of those only the marked strips: what it
// skips would add nothing to any gradient.  The forward pass stores every
// 64-position round of its walk in which it marked something, so every
// mark of the pass is in place; other bytes keep what they held, and a
// stale mark only makes the backward evaluate a strip in full, with the
// same result.  The backward reads a block's bytes only up to that block's
// last blended entry.
constexpr int kMarkKeep = 32;   // rounds of a forward walk whose marks are staged in LDS

struct Marks {
  uint8_t* base;   // plane f (forward wavefront f of a tile) at base + f * cap; null: no marks
  uint64_t cap;    // positions per plane: a tile is marked iff its list ends at or before cap
  uint64_t* tag;   // the forward pass stores `key` here; the backward trusts the planes iff it matches
  uint64_t key;
};

__device__ __forceinline__ Record load_record(const Record* __restrict__ rec, uint32_t id) {
  return rec[id];
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xf, true));
}

// Sums of the 12 record-gradient terms over the 64 lanes, as a
// reduce-scatter: exchanging half of the values with the lane one apart
// (then two apart) leaves each lane with 3 partial sums of its own terms,
// q = 6 (lane & 1) + 3 ((lane >> 1) & 1) + i; those are summed over the 16
// lanes sharing lane & 3 (row rotations by 4 and 8, then the gfx950 row and
// half swaps).  Lanes 0..3 end up holding all 12 totals, 45 VALU operations
// in place of 72 for twelve full reductions.
__device__ __forceinline__ float swap_sum16(float v) {
  const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
__device__ __forceinline__ float swap_sum32(float v) {
  const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
__device__ __forceinline__ void wave_reduce12(const float* g, int lane, float* out3) {
  const bool b0 = (lane & 1) != 0, b1 = (lane & 2) != 0;
  float h[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float send = b0 ? g[i] : g[i + 6];
    const float keep = b0 ? g[i + 6] : g[i];
    h[i] = keep + dpp<0xb1, 0xf>(send);      // quad_perm [1,0,3,2]
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float send = b1 ? h[i] : h[i + 3];
    const float keep = b1 ? h[i + 3] : h[i];
    float v = keep + dpp<0x4e, 0xf>(send);   // quad_perm [2,3,0,1]
    v += dpp<0x124, 0xf>(v);                 // row_ror:4
    v += dpp<0x128, 0xf>(v);                 // row_ror:8
    v = swap_sum16(v);
    out3[i] = swap_sum32(v);
  }
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int o = __shfl_xor(v, m, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Uniform over the wavefront (the compiler cannot always prove it).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A wave-uniform value copied once into a vector register, so that the
// per-strip instructions that also read a scalar operand (one scalar source
// per vector instruction) take it without a copy at every use.
__device__ __forceinline__ float in_vgpr(float v) {
  asm("" : "+v"(v));
  return v;
}
__device__ __forceinline__ int in_vgpr(int v) {
  asm("" : "+v"(v));
  return v;
}

// One wavefront's block of pixels (sub-block `wave` of `tile`), front to back.
// Per record, everything that does not depend on the lane is decided once
// for the wavefront on lane masks (rect against each strip, pixels still
// open, any pair reaching alpha_min, d_o == 0); the per-pixel updates are
// selects on a mask, so the lanes never branch apart.
template <int T, int IPL, bool DEPTH>
__device__ __forceinline__ void fwd_block(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const CamPack& cp, const Opts& o, float* __restrict__ img,
    float* __restrict__ T_final, int32_t* __restrict__ last_idx, int32_t* __restrict__ n_contrib,
    float* __restrict__ depth, const Marks& mk, uint32_t tile, int wave, int lane) {
  using Gm = Geometry<T>;
  constexpr int PPL = Gm::PPL;
  constexpr int RS = Gm::ROWSTEP;
  if (tile >= cp.tiles_total) return;  // never index past the tile arrays
  const int c = cam_of_tile(cp, tile);
  const CamDev& cam = cp.cam[c];
  const uint32_t lt = tile - cam.tile_off;
  const int ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int tx = (int)(lt - (uint32_t)ty * (uint32_t)cam.tiles_x);
  const int ox = uniform(tx * T + (wave % (T / Gm::SUB)) * Gm::SUB);
  const int oy = uniform(ty * T + (wave / (T / Gm::SUB)) * Gm::SUB);
  const int px = ox + lane % Gm::SUB;
  const float fpx = (float)px + 0.5f;
  const int py0 = oy + lane / Gm::SUB;
  float Tr[PPL], C0[PPL], C1[PPL], C2[PPL], Dz[PPL];
  int32_t cnt[PPL], last[PPL];
  uint64_t open[PPL];   // lanes whose pixel j still takes entries
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    Tr[j] = 1.0f;
    C0[j] = C1[j] = C2[j] = Dz[j] = 0.0f;
    cnt[j] = 0;
    last[j] = -1;
    open[j] = lanes(px < cam.width && py0 + j * RS < cam.height);
  }
  // the tile's list; positions below are indices into it (fit int32: a
  // list holds at most one entry per record)
  const uint32_t* __restrict__ lst = vals + ranges[2 * tile];
  const int64_t len = (int64_t)ranges[2 * tile + 1] - (int64_t)ranges[2 * tile];
  // this wavefront's mark plane, from the tile's list start (none when the
  // list ends beyond the planes)
  uint8_t* __restrict__ marks = nullptr;
  if (mk.base != nullptr && (uint64_t)ranges[2 * tile + 1] <= mk.cap)
    marks = mk.base + (uint64_t)wave * mk.cap + ranges[2 * tile];
  // the marks of the walk's first kMarkKeep rounds wait in LDS until the
  // walk ends (a walk is a few rounds: pixels end at T_min soon after their
  // last blended entries); rounds past those are marked in full (0xff: the
  // backward evaluates every strip there, with the same result).  Stored
  // round by round they would stall the walk: the entry loop waits for
  // every vector memory operation in flight, stores included.
  __shared__ uint8_t s_marks[Gm::WAVES][kMarkKeep * 64];
  uint8_t* s_mk = s_marks[wave];
  int walked = 0;   // rounds walked
  const float amin = o.alpha_min, amax = o.alpha_max, tmin = o.t_min;
  const float l2amin = __builtin_amdgcn_logf(amin);
  const float e39 = erfc_fast(3.9f);
  uint64_t any_open = 0ull;
#pragma unroll
  for (int j = 0; j < PPL; ++j) any_open |= open[j];

  for (int64_t base = 0; any_open != 0ull && base < len; base += 64 * IPL) {
    uint32_t ids[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int64_t p = base + k * 64 + lane;
      ids[k] = p < len ? lst[p] : 0u;
    }
    const int64_t nb = (len - base) < (int64_t)(64 * IPL) ? (len - base) : (int64_t)(64 * IPL);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int lim = (int)nb - k * 64;
      if (lim <= 0 || any_open == 0ull) break;
      const int cntk = lim < 64 ? lim : 64;
      uint32_t mark = 0u;   // lane l: the strips that took entry l of this round
      for (int l = 0; l < cntk && any_open != 0ull; ++l) {
        const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)ids[k], l);
        const Record r = load_record(rec, id);
        // the whole record in one request: nearly every listed entry meets
        // the block's columns, so loading the rect first and the rest only
        // after the column test costs a second round trip almost always
        asm volatile("" ::"s"(r.mx), "s"(r.my), "s"(r.kx), "s"(r.ky), "s"(r.qa), "s"(r.qb), "s"(r.qc),
                     "s"(r.alpha2), "s"(r.r), "s"(r.g), "s"(r.b), "s"(r.d_o), "s"(r.xr), "s"(r.yr));
        const int x0 = (int)(r.xr & 0xffffu), x1 = (int)(r.xr >> 16);
        const int y0 = (int)(r.yr & 0xffffu), y1 = (int)(r.yr >> 16);
        const uint64_t cols = lanes(px >= x0) & lanes(px <= x1);
        if (cols == 0ull) continue;
        const int32_t pos = (int32_t)(base + k * 64 + l);
        uint32_t strips = 0u;
        const int32_t posv = in_vgpr(pos);
        const float a2v = in_vgpr(r.alpha2);
        const RecordU u = record_uniform(r, x0, y0, y1, l2amin);
        const Column col = column_of(r, u, fpx);
        const float p2c = r.qc * (-0.5f * kLog2e);
        bool ended = false;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          const float fpy = (float)(py0 + j * RS) + 0.5f;
          uint64_t m = open[j] & cols & lanes(fpy > u.y0f) & lanes(fpy < u.y1p);
          if (m == 0ull) continue;
          const float dy = (fpy - u.y0f) - r.my;
          const float p2 = gauss_p2(col, p2c, dy);
          m &= lanes(!(p2 > 0.0f)) & lanes(!(p2 < u.p2_min));
          if (m == 0ull) continue;
          const float G = __builtin_amdgcn_exp2f(p2);
          m &= lanes(!(G * u.hb < amin));
          if (m == 0ull) continue;
          const float I = half_factor(r, u, col, dy, m, e39);
          const float a = clamp_alpha(fmaf(r.d_o, I, a2v) * G, amax);
          m &= lanes(!(a < amin));
          if (m == 0ull) continue;
          strips |= 1u << j;   // a superset of the strips that blend it (a stopping pixel does not)
          const float Tn = Tr[j] * (1.0f - a);
          const uint64_t stop = m & lanes(Tn < tmin);
          const bool take = in_mask(m & ~stop);
          const float w = take ? a * Tr[j] : 0.0f;
          C0[j] = fmaf(r.r, w, C0[j]);
          C1[j] = fmaf(r.g, w, C1[j]);
          C2[j] = fmaf(r.b, w, C2[j]);
          if constexpr (DEPTH) Dz[j] = fmaf(__uint_as_float(r.depth), w, Dz[j]);
          Tr[j] = take ? Tn : Tr[j];
          cnt[j] += take ? 1 : 0;
          last[j] = take ? posv : last[j];
          open[j] &= ~stop;
          ended |= stop != 0ull;
        }
        if (marks) mark = lane == l ? strips : mark;
        if (ended) {
          any_open = 0ull;
#pragma unroll
          for (int j = 0; j < PPL; ++j) any_open |= open[j];
        }
      }
      if (marks) {
        const int r = (int)(base >> 6) + k;
        walked = r + 1;
        if (r < kMarkKeep) s_mk[r * 64 + lane] = (uint8_t)mark;
      }
    }
  }
  if (marks) {
    for (int r = 0; r < walked; ++r) {
      const int64_t p = (int64_t)r * 64 + lane;
      if (p < len) marks[p] = r < kMarkKeep ? s_mk[r * 64 + lane] : (uint8_t)0xffu;
    }
  }
  const uint64_t plane = (uint64_t)cam.width * cam.height;
  float* im = img + 3 * cam.pix_off;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int py = py0 + j * RS;
    if (!(px < cam.width && py < cam.height)) continue;
    const uint64_t pix = (uint64_t)py * cam.width + px;
    im[pix] = fmaf(Tr[j], o.bg[0], C0[j]);
    im[plane + pix] = fmaf(Tr[j], o.bg[1], C1[j]);
    im[2 * plane + pix] = fmaf(Tr[j], o.bg[2], C2[j]);
    T_final[cam.pix_off + pix] = Tr[j];
    last_idx[cam.pix_off + pix] = last[j];
    n_contrib[cam.pix_off + pix] = cnt[j];
    if constexpr (DEPTH) depth[cam.pix_off + pix] = Dz[j];
  }
}

// Tile of launch slot b in the per-tile backward grid, placed for the eight
// XCDs (each with its own L2).  Workgroups go to the XCDs in turn, so slots
// x + 32 m + 8 j (j < 4) all run on XCD x; they take positions
// 4 (x + 8 m) + j of the tiles in block order (each camera's tiles by 2x2
// blocks: block rows of two tile rows, blocks left to right, row-major inside
// a block; a last odd row or column gives narrower blocks).  The tiles of a
// block, which share most of their records, are thus read through one L2,
// and consecutive blocks still spread over all XCDs.  Slots from 32 (n / 32)
// on take their own position.  Both steps are bijections of [0, n).
__device__ __forceinline__ uint32_t xcd_block_tile(uint32_t b, const CamPack& cp) {
  const uint32_t full = cp.tiles_total / 32u * 32u;
  const uint32_t p = b < full ? 4u * ((b % 8u) + 8u * (b / 32u)) + (b / 8u) % 4u : b;
  const int c = cam_of_tile(cp, p);
  const CamDev& cam = cp.cam[c];
  const uint32_t tx = (uint32_t)cam.tiles_x, ty = (uint32_t)cam.tiles_y;
  const uint32_t lp = p - cam.tile_off;
  const uint32_t br = lp / (2u * tx), pr = lp - br * 2u * tx;   // block row, position in it
  const uint32_t h = ty - 2u * br < 2u ? ty - 2u * br : 2u;      // its height (1 or 2)
  const uint32_t bc = pr / (2u * h), in = pr - bc * 2u * h;      // block, position in it
  uint32_t col, row;
  if (2u * bc + 1u < tx) {           // two columns wide
    col = 2u * bc + in % 2u;
    row = 2u * br + in / 2u;
  } else {                           // the last, one-column block
    col = 2u * bc;
    row = 2u * br + in;
  }
  return cam.tile_off + row * tx + col;
}

// Next tile rank of a persistent workgroup (all its wavefronts see it).
__device__ __forceinline__ uint32_t next_tile(uint32_t* counter, uint32_t* s_w) {
  __syncthreads();   // every wavefront has read the previous rank
  if (threadIdx.x == 0) *s_w = atomicAdd(counter, 1u);
  __syncthreads();
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)*s_w);
}

// Eight wavefronts per SIMD (at most 64 VGPRs) where the kernel needs
// barely more: the walk is latency-bound and loses more with one wavefront
// fewer than with the two registers it then spills.  Instantiations that
// would spill more (the depth output, 512-entry rounds) are left alone; the
// persistent form keeps six (at most 80 VGPRs, no spill).
template <int T, int IPL, bool DEPTH>
constexpr int kFwdMinWaves = (!DEPTH && IPL <= 4) ? 8 : 1;

template <int T, int IPL, bool DEPTH>
__global__ __launch_bounds__(64 * Geometry<T>::WAVES) __attribute__((amdgpu_waves_per_eu(kFwdMinWaves<T, IPL, DEPTH>))) void
render_fwd_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, CamPack cp, Opts o, float* __restrict__ img,
    float* __restrict__ T_final, int32_t* __restrict__ last_idx, int32_t* __restrict__ n_contrib,
    float* __restrict__ depth, Marks mk) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *mk.tag = mk.key;
  fwd_block<T, IPL, DEPTH>(rec, vals, ranges, cp, o, img, T_final, last_idx, n_contrib, depth, mk, blockIdx.x,
                           threadIdx.x >> 6, threadIdx.x & 63);
}

// Persistent form: workgroups of one tile's wavefronts (they share the
// tile's records through the CU's scalar cache), a grid sized to the chip;
// every workgroup takes tiles from a counter in `order` (longest list
// first) so that long tiles do not start last.
template <int T, int IPL, bool DEPTH>
__global__ __launch_bounds__(64 * Geometry<T>::WAVES) __attribute__((amdgpu_waves_per_eu(kFwdMinWaves<T, IPL, DEPTH> == 8 ? 6 : 1))) void
render_fwd_persistent_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, CamPack cp, Opts o,
    float* __restrict__ img, float* __restrict__ T_final, int32_t* __restrict__ last_idx,
    int32_t* __restrict__ n_contrib, float* __restrict__ depth, Marks mk, uint32_t* __restrict__ counter) {
  __shared__ uint32_t s_w;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && threadIdx.x == 0) *mk.tag = mk.key;
  for (uint32_t w = next_tile(counter, &s_w); w < cp.tiles_total; w = next_tile(counter, &s_w))
    fwd_block<T, IPL, DEPTH>(rec, vals, ranges, cp, o, img, T_final, last_idx, n_contrib, depth, mk, order[w],
                             wave, lane);
}

// One wavefront's block of pixels, back to front.  Same masks as the
// forward pass; a pixel takes part in an entry only at or before its last
// blended one, and the state of the other lanes is kept by selects (their
// gradient terms are exact zeros).
template <int T, int IPL>
__device__ __forceinline__ void bwd_block(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const CamPack& cp, const Opts& o,
    const float* __restrict__ T_final, const int32_t* __restrict__ last_idx,
    const float* __restrict__ dL_dimg, float* __restrict__ rgrad, const Marks& mk, bool marked,
    uint32_t tile, int wave, int lane) {
  using Gm = BwdGeometry<T>;
  using Gf = Geometry<T>;
  constexpr int PPL = Gm::PPL;
  constexpr int RS = Gm::ROWSTEP;
  // the block is SPLIT forward blocks stacked vertically, each of FPPL strips
  constexpr int SPLIT = Gm::SUBY / Gf::SUB;
  constexpr int FPPL = Gf::PPL;
  static_assert(Gm::SUBX == Gf::SUB && RS == Gf::ROWSTEP && PPL == SPLIT * FPPL,
                "backward strips are the forward blocks' strips");
  if (tile >= cp.tiles_total) return;  // never index past the tile arrays
  const int c = cam_of_tile(cp, tile);
  const CamDev& cam = cp.cam[c];
  const uint32_t lt = tile - cam.tile_off;
  const int ty = (int)(lt / (uint32_t)cam.tiles_x);
  const int tx = (int)(lt - (uint32_t)ty * (uint32_t)cam.tiles_x);
  const int ox = uniform(tx * T + (wave % (T / Gm::SUBX)) * Gm::SUBX);
  const int oy = uniform(ty * T + (wave / (T / Gm::SUBX)) * Gm::SUBY);
  const int px = ox + lane % Gm::SUBX;
  const float fpx = (float)px + 0.5f;
  const int py0 = oy + lane / Gm::SUBX;
  const uint64_t plane = (uint64_t)cam.width * cam.height;
  const float* g = dL_dimg + 3 * cam.pix_off;

  int32_t last[PPL], top_j[PPL];
  float Tr[PPL], dL0[PPL], dL1[PPL], dL2[PPL];
  // S: the colour of the entries behind the current one (already replayed),
  // dotted with dL/dcolour -- the only way that colour enters dL/dalpha
  float S[PPL], tbg[PPL];
  int top = -1;
#pragma unroll
  for (int j = 0; j < PPL; ++j) {
    const int py = py0 + j * RS;
    const bool inside = px < cam.width && py < cam.height;
    last[j] = -1;
    float Tf = 1.0f;
    dL0[j] = dL1[j] = dL2[j] = 0.0f;
    if (inside) {
      const uint64_t pix = (uint64_t)py * cam.width + px;
      Tf = T_final[cam.pix_off + pix];
      last[j] = last_idx[cam.pix_off + pix];
      dL0[j] = g[pix];
      dL1[j] = g[plane + pix];
      dL2[j] = g[2 * plane + pix];
    }
    Tr[j] = Tf;
    S[j] = 0.0f;
    // the background seen through the final transmittance: its share of
    // dL/dalpha is -T_final / (1 - alpha) * (bg . dL)
    tbg[j] = -Tf * (o.bg[0] * dL0[j] + o.bg[1] * dL1[j] + o.bg[2] * dL2[j]);
    top_j[j] = uniform(wave_max(last[j]));   // last entry any pixel of strip j blended
    top = top_j[j] > top ? top_j[j] : top;
  }
  if (top < 0) return;
  const uint32_t* __restrict__ lst = vals + ranges[2 * tile];
  const float amin = o.alpha_min, amax = o.alpha_max;
  const float l2amin = __builtin_amdgcn_logf(amin);
  const float e39 = erfc_fast(3.9f);
  // the mark planes of the forward blocks, each read up to that block's
  // last blended entry
  marked = marked && (uint64_t)ranges[2 * tile + 1] <= mk.cap;
  const uint8_t* mplane[SPLIT];
  int32_t mtop[SPLIT];
#pragma unroll
  for (int q = 0; q < SPLIT; ++q) {
    const int fw = ((wave / (T / Gm::SUBX)) * SPLIT + q) * (T / Gf::SUB) + wave % (T / Gm::SUBX);
    mplane[q] = marked ? mk.base + (uint64_t)fw * mk.cap + ranges[2 * tile] : nullptr;
    mtop[q] = -1;
#pragma unroll
    for (int j = q * FPPL; j < (q + 1) * FPPL; ++j) mtop[q] = top_j[j] > mtop[q] ? top_j[j] : mtop[q];
  }

  // list indices top, top-1, ..., 0 in rounds of 64 * IPL
  for (int32_t hi = top; hi >= 0; hi -= 64 * IPL) {
    uint32_t ids[IPL], sm[IPL];   // entry ids and their strip marks (all strips when unmarked)
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int32_t p = hi - (k * 64 + lane);
      ids[k] = p >= 0 ? lst[p] : 0u;
      sm[k] = 0u;
      if (p >= 0) {
        if (marked) {
#pragma unroll
          for (int q = 0; q < SPLIT; ++q)
            if (p <= mtop[q]) sm[k] |= (uint32_t)mplane[q][p] << (q * FPPL);
        } else {
          sm[k] = (1u << PPL) - 1u;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      if (hi - k * 64 < 0) break;
      // the round's ids are waited for here, once: the entry loop issues
      // float atomics, and a load still pending at its head would make
      // every entry wait for all memory operations in flight, the previous
      // entry's atomics included
      asm volatile("" ::"v"(ids[k]));
      // the marked entries of the round, in list order back to front
      for (uint64_t todo = lanes(sm[k] != 0u); todo != 0ull; todo &= todo - 1ull) {
        const int l = (int)__builtin_ctzll(todo);
        const uint32_t strips = (uint32_t)__builtin_amdgcn_readlane((int)sm[k], l);
        const uint32_t id = (uint32_t)__builtin_amdgcn_readlane((int)ids[k], l);
        const Record r = load_record(rec, id);
        // the whole record in one request: nearly every listed entry meets
        // the block's columns, so loading the rect first and the rest only
        // after the column test costs a second round trip almost always
        asm volatile("" ::"s"(r.mx), "s"(r.my), "s"(r.kx), "s"(r.ky), "s"(r.qa), "s"(r.qb), "s"(r.qc),
                     "s"(r.alpha2), "s"(r.r), "s"(r.g), "s"(r.b), "s"(r.d_o), "s"(r.xr), "s"(r.yr));
        const int x0 = (int)(r.xr & 0xffffu), x1 = (int)(r.xr >> 16);
        const int y0 = (int)(r.yr & 0xffffu), y1 = (int)(r.yr >> 16);
        const uint64_t cols = lanes(px >= x0) & lanes(px <= x1);
        if (cols == 0ull) continue;
        const int32_t pos = hi - (k * 64 + l);
        const float a2v = in_vgpr(r.alpha2);
        const float cdu = r.d_o * kTwoOverSqrtPi;   // d(d_o I)/du = d_o 2/sqrt(pi) exp(-u^2)
        const RecordU u = record_uniform(r, x0, y0, y1, l2amin);
        const Column col = column_of(r, u, fpx);
        const float p2c = r.qc * (-0.5f * kLog2e);
        // per-lane sums over the lane's pixels: the centre, conic and
        // half-factor gradients are linear in them (the lane's pixels share
        // the column offset dx), so they are formed once per entry below
        float sGG = 0.0f, sT = 0.0f, sT2 = 0.0f, sDu = 0.0f, sDuDy = 0.0f;   // sums of GG, GG dy, GG dy^2, du, du dy
        float g7 = 0.0f, g8 = 0.0f, g9 = 0.0f, g10 = 0.0f, g11 = 0.0f;
        bool any = false;
#pragma unroll
        for (int j = 0; j < PPL; ++j) {
          if (pos > top_j[j] || ((strips >> j) & 1u) == 0u) continue;
          const float fpy = (float)(py0 + j * RS) + 0.5f;
          uint64_t m = cols & lanes(fpy > u.y0f) & lanes(fpy < u.y1p) & lanes(pos <= last[j]);
          if (m == 0ull) continue;
          const float dy = (fpy - u.y0f) - r.my;
          const float p2 = gauss_p2(col, p2c, dy);
          m &= lanes(!(p2 > 0.0f)) & lanes(!(p2 < u.p2_min));
          if (m == 0ull) continue;
          const float G = __builtin_amdgcn_exp2f(p2);
          m &= lanes(!(G * u.hb < amin));
          if (m == 0ull) continue;
          const float I = half_factor(r, u, col, dy, m, e39);
          const float hgf = fmaf(r.d_o, I, a2v);
          const float HG = hgf * G;
          const float a = clamp_alpha(HG, amax);
          m &= lanes(!(a < amin));
          if (m == 0ull) continue;
          any = true;
          {
            // gradient arithmetic only (every decision is taken above): the
            // compiler may fuse multiply-adds here
#pragma clang fp contract(fast)
            const bool on = in_mask(m);
            const float inv1ma = __builtin_amdgcn_rcpf(1.0f - a);  // 1 - a >= 1 - alpha_max
            const float Tb = Tr[j] * inv1ma;
            const float aon = on ? a : 0.0f;
            const float wcol = aon * Tb;
            g9 += wcol * dL0[j];
            g10 += wcol * dL1[j];
            g11 += wcol * dL2[j];
            // dL/dalpha = T (c - A) . dL - T_final / (1 - alpha) bg . dL,
            // A the colour behind: (c . dL - S) T
            const float cdl = r.r * dL0[j] + r.g * dL1[j] + r.b * dL2[j];
            const float dcs = cdl - S[j];
            const float dLda = dcs * Tb + inv1ma * tbg[j];
            S[j] = fmaf(aon, dcs, S[j]);
            Tr[j] = on ? Tb : Tr[j];
            // no gradient through the alpha_max clamp
            const float dHG = in_mask(m & lanes(!(HG > amax))) ? dLda : 0.0f;
            const float dHGG = dHG * G;
            g7 += dHGG;
            g8 += dHGG * I;
            float du = 0.0f;
            if (u.split) {
              const float w = fmaf(r.ky, dy, col.kxdx);
              du = (dHGG * cdu) * __builtin_amdgcn_exp2f(-kLog2e * w * w);
            }
            sDu += du;
            sDuDy += du * dy;
            const float GG = dHG * hgf * G;   // dL/dG times G
            const float t = GG * dy;
            sGG += GG;
            sT += t;
            sT2 += t * dy;
          }
        }
        if (!any) continue;
        float gs[HGS_RECORD_GRAD_FLOATS];
        {
#pragma clang fp contract(fast)
          gs[0] = col.qadx * sGG + r.qb * sT - r.kx * sDu;
          gs[1] = col.qbdx * sGG + r.qc * sT - r.ky * sDu;
          gs[2] = -0.5f * col.dx * col.dx * sGG;
          gs[3] = -col.dx * sT;
          gs[4] = -0.5f * sT2;
          gs[5] = col.dx * sDu;
          gs[6] = sDuDy;
          gs[7] = g7;
          gs[8] = g8;
          gs[9] = g9;
          gs[10] = g10;
          gs[11] = g11;
        }
        float tot[3];
        wave_reduce12(gs, lane, tot);
        if (lane < 4) {
          float* dst = rgrad + (uint64_t)id * HGS_RECORD_GRAD_FLOATS + 6 * (lane & 1) + 3 * (lane >> 1);
#pragma unroll
          for (int i = 0; i < 3; ++i)
            if (tot[i] != 0.0f) atomicAdd(dst + i, tot[i]);
        }
      }
    }
  }
}

template <int T, int IPL>
__global__ __launch_bounds__(64 * BwdGeometry<T>::WAVES) void render_bwd_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, CamPack cp, Opts o, const float* __restrict__ T_final,
    const int32_t* __restrict__ last_idx, const float* __restrict__ dL_dimg,
    float* __restrict__ rgrad, Marks mk) {
  const bool marked = mk.base != nullptr && *mk.tag == mk.key;
  bwd_block<T, IPL>(rec, vals, ranges, cp, o, T_final, last_idx, dL_dimg, rgrad, mk, marked,
                    xcd_block_tile(blockIdx.x, cp), threadIdx.x >> 6, threadIdx.x & 63);
}

template <int T, int IPL>
__global__ __launch_bounds__(64 * BwdGeometry<T>::WAVES) __attribute__((amdgpu_waves_per_eu(4))) void
render_bwd_persistent_kernel(
    const Record* __restrict__ rec, const uint32_t* __restrict__ vals,
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ order, CamPack cp, Opts o,
    const float* __restrict__ T_final, const int32_t* __restrict__ last_idx,
    const float* __restrict__ dL_dimg, float* __restrict__ rgrad, Marks mk, uint32_t* __restrict__ counter) {
  __shared__ uint32_t s_w;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool marked = mk.base != nullptr && *mk.tag == mk.key;
  for (uint32_t w = next_tile(counter, &s_w); w < cp.tiles_total; w = next_tile(counter, &s_w))
    bwd_block<T, IPL>(rec, vals, ranges, cp, o, T_final, last_idx, dL_dimg, rgrad, mk, marked, order[w], wave,
                      lane);
}

__global__ void clear_counter_kernel(uint32_t* __restrict__ p) { *p = 0u; }

__global__ void zero_f32_kernel(float* __restrict__ p, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = t; i < n; i += stride) p[i] = 0.0f;
}

// Workgroups of the persistent grid: as many workgroups of `threads` as
// the chip keeps resident, never more than there are work items.
template <typename F>
unsigned persistent_grid(F kernel, uint32_t n_work, int threads) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
    per_cu = 8;
  const uint64_t g = (uint64_t)cus * (uint64_t)per_cu;
  return (unsigned)(g < n_work ? g : (n_work > 0 ? n_work : 1));
}

template <int T, int B, bool DEPTH>
hipError_t fwd_launch_d(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                        const uint32_t* order, const CamPack& cp, const Opts& o, float* img, float* Tf,
                        int32_t* li, int32_t* nc, float* depth, void* ws, const Marks& mk, hipStream_t s) {
  if (order) {
    uint32_t* counter = static_cast<uint32_t*>(ws);
    hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    constexpr int threads = 64 * Geometry<T>::WAVES;
    hipLaunchKernelGGL((render_fwd_persistent_kernel<T, B / 64, DEPTH>),
                       dim3(persistent_grid(render_fwd_persistent_kernel<T, B / 64, DEPTH>, cp.tiles_total,
                                            threads)),
                       dim3(threads), 0, s, rec, vals, ranges, order, cp, o, img, Tf, li, nc, depth, mk, counter);
  } else {
    hipLaunchKernelGGL((render_fwd_kernel<T, B / 64, DEPTH>), dim3(cp.tiles_total),
                       dim3(64 * Geometry<T>::WAVES), 0, s, rec, vals, ranges, cp, o, img, Tf, li, nc, depth, mk);
  }
  return hipGetLastError();
}

template <int T, int B>
hipError_t fwd_launch(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                      const uint32_t* order, const CamPack& cp, const Opts& o, float* img, float* Tf,
                      int32_t* li, int32_t* nc, float* depth, void* ws, const Marks& mk, hipStream_t s) {
  return depth ? fwd_launch_d<T, B, true>(rec, vals, ranges, order, cp, o, img, Tf, li, nc, depth, ws, mk, s)
               : fwd_launch_d<T, B, false>(rec, vals, ranges, order, cp, o, img, Tf, li, nc, depth, ws, mk, s);
}

template <int T, int B>
hipError_t bwd_launch(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                      const uint32_t* order, const CamPack& cp, const Opts& o, const float* Tf,
                      const int32_t* li, const float* dL, float* rg, void* ws, const Marks& mk, hipStream_t s) {
  if (order) {
    uint32_t* counter = static_cast<uint32_t*>(ws) + 1;
    hipLaunchKernelGGL(clear_counter_kernel, dim3(1), dim3(1), 0, s, counter);
    constexpr int threads = 64 * BwdGeometry<T>::WAVES;
    hipLaunchKernelGGL((render_bwd_persistent_kernel<T, B / 64>),
                       dim3(persistent_grid(render_bwd_persistent_kernel<T, B / 64>, cp.tiles_total, threads)),
                       dim3(threads), 0, s, rec, vals, ranges, order, cp, o, Tf, li, dL, rg, mk, counter);
  } else {
    hipLaunchKernelGGL((render_bwd_kernel<T, B / 64>), dim3(cp.tiles_total), dim3(64 * BwdGeometry<T>::WAVES),
                       0, s, rec, vals, ranges, cp, o, Tf, li, dL, rg, mk);
  }
  return hipGetLastError();
}

// Render workspace: [0, 256) the persistent rasters' work counters (u32 [0]
// forward, [1] backward) and at byte 64 the mark tag; from 256 on, the mark
// planes (one per forward wavefront of a tile, `cap` bytes each).
constexpr size_t kRenderWsHead = 256;
constexpr size_t kMarkTagOffset = 64;

int mark_planes(int tile) { return tile == 32 ? Geometry<32>::WAVES : (tile == 16 ? Geometry<16>::WAVES : Geometry<8>::WAVES); }

// The planes a workspace of ws_bytes holds, and the key that ties them to
// these lists: the forward pass stores it, the backward compares it, so a
// backward given another workspace (or one of another size) than its
// forward pass ignores the planes instead of trusting stale marks.
Marks make_marks(const uint32_t* vals, const uint32_t* ranges, const CamPack& cp, const Opts& o, void* ws,
                 size_t ws_bytes) {
  Marks mk;
  const uint64_t planes = (uint64_t)mark_planes(o.tile);
  mk.cap = ws_bytes > kRenderWsHead ? (uint64_t)(ws_bytes - kRenderWsHead) / planes : 0u;
  mk.base = mk.cap > 0 ? static_cast<uint8_t*>(ws) + kRenderWsHead : nullptr;
  mk.tag = reinterpret_cast<uint64_t*>(static_cast<char*>(ws) + kMarkTagOffset);
  // splitmix64 over the list buffers, the plane size and the tiling
  uint64_t z = (uint64_t)(uintptr_t)vals ^ ((uint64_t)(uintptr_t)ranges << 1) ^ (mk.cap * 0x9e3779b97f4a7c15ull) ^
               ((uint64_t)cp.tiles_total << 40) ^ ((uint64_t)o.tile << 56) ^ 0x6867735f6d61726bull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  mk.key = z != 0u ? z : 1u;
  return mk;
}

// Normals estimated from the accumulated depth (see launch_depth_normals).
__global__ __launch_bounds__(256) void depth_normals_kernel(const float* __restrict__ depth,
                                                            const float* __restrict__ T_final, CamPack cp,
                                                            uint64_t n_pix, float* __restrict__ normals) {
  const uint64_t p = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n_pix) return;
  int c = 0;
  for (int i = 1; i < cp.n_cams; ++i)
    if (p >= cp.cam[i].pix_off) c = i;
  const CamDev& cam = cp.cam[c];
  const int W = cam.width, H = cam.height;
  const uint64_t local = p - cam.pix_off;
  const int v = (int)(local / (uint64_t)W), u = (int)(local - (uint64_t)v * W);
  const float* D = depth + cam.pix_off;
  const float* Tf = T_final + cam.pix_off;
  double n0 = 0.0, n1 = 0.0, n2 = 0.0;
  if (u >= 1 && u < W - 1 && v >= 1 && v < H - 1) {
    const int du[4] = {1, -1, 0, 0}, dv[4] = {0, 0, 1, -1};
    double P[4][3];
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint64_t pq = (uint64_t)(v + dv[q]) * W + (u + du[q]);
      const double acc = 1.0 - (double)Tf[pq];
      ok = ok && acc > 0.0;
      const double d = acc > 0.0 ? (double)D[pq] / acc : 0.0;
      P[q][0] = d * (((double)(u + du[q]) + 0.5 - (double)cam.cx) / (double)cam.fx);
      P[q][1] = d * (((double)(v + dv[q]) + 0.5 - (double)cam.cy) / (double)cam.fy);
      P[q][2] = d;
    }
    if (ok) {
      const double ax = P[0][0] - P[1][0], ay = P[0][1] - P[1][1], az = P[0][2] - P[1][2];
      const double bx = P[2][0] - P[3][0], by = P[2][1] - P[3][1], bz = P[2][2] - P[3][2];
      const double cx = -(ay * bz - az * by), cy = -(az * bx - ax * bz), cz = -(ax * by - ay * bx);
      const double nn = sqrt(cx * cx + cy * cy + cz * cz);
      if (nn > 0.0) {
        n0 = cx / nn;
        n1 = cy / nn;
        n2 = cz / nn;
      }
    }
  }
  float* out = normals + 3 * cam.pix_off;
  const uint64_t plane = (uint64_t)W * H;
  out[local] = (float)n0;
  out[plane + local] = (float)n1;
  out[2 * plane + local] = (float)n2;
}

#define HGS_DISPATCH(T_, B_, CALL) \
  if (o.tile == T_ && o.batch == B_) return CALL<T_, B_>

}  // namespace

size_t render_workspace_bytes() { return kRenderWsHead; }

size_t render_workspace_bytes(int tile, int64_t capacity) {
  if (capacity <= 0) return kRenderWsHead;
  const uint64_t planes = (uint64_t)(mark_planes(tile) * capacity);
  return kRenderWsHead + (size_t)((planes + 255u) / 256u * 256u);
}

hipError_t launch_render_fwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const uint32_t* tile_order, const CamPack& cp, const Opts& o,
                             float* img, float* T_final, int32_t* last_idx, int32_t* n_contrib,
                             float* depth, void* ws, size_t ws_bytes, hipStream_t s) {
  if (cp.tiles_total == 0) return hipSuccess;
  const Marks mk = make_marks(vals, ranges, cp, o, ws, ws_bytes);
#define ARGS (rec, vals, ranges, tile_order, cp, o, img, T_final, last_idx, n_contrib, depth, ws, mk, s)
  HGS_DISPATCH(8, 128, fwd_launch) ARGS;
  HGS_DISPATCH(8, 256, fwd_launch) ARGS;
  HGS_DISPATCH(8, 512, fwd_launch) ARGS;
  HGS_DISPATCH(16, 128, fwd_launch) ARGS;
  HGS_DISPATCH(16, 256, fwd_launch) ARGS;
  HGS_DISPATCH(16, 512, fwd_launch) ARGS;
  HGS_DISPATCH(32, 128, fwd_launch) ARGS;
  HGS_DISPATCH(32, 256, fwd_launch) ARGS;
  HGS_DISPATCH(32, 512, fwd_launch) ARGS;
#undef ARGS
  return hipErrorInvalidValue;
}

hipError_t launch_zero_f32(float* p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + 255) / 256;
  g = g < 1 ? 1 : (g > 8192 ? 8192 : g);
  hipLaunchKernelGGL(zero_f32_kernel, dim3((unsigned)g), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_render_bwd(const Record* rec, const uint32_t* vals, const uint32_t* ranges,
                             const uint32_t* tile_order, const CamPack& cp, const Opts& o,
                             const float* T_final, const int32_t* last_idx, const float* dL_dimg,
                             float* rec_grads, void* ws, size_t ws_bytes, hipStream_t s) {
  if (cp.tiles_total == 0) return hipSuccess;
  const Marks mk = make_marks(vals, ranges, cp, o, ws, ws_bytes);
#define ARGS (rec, vals, ranges, tile_order, cp, o, T_final, last_idx, dL_dimg, rec_grads, ws, mk, s)
  HGS_DISPATCH(8, 128, bwd_launch) ARGS;
  HGS_DISPATCH(8, 256, bwd_launch) ARGS;
  HGS_DISPATCH(8, 512, bwd_launch) ARGS;
  HGS_DISPATCH(16, 128, bwd_launch) ARGS;
  HGS_DISPATCH(16, 256, bwd_launch) ARGS;
  HGS_DISPATCH(16, 512, bwd_launch) ARGS;
  HGS_DISPATCH(32, 128, bwd_launch) ARGS;
  HGS_DISPATCH(32, 256, bwd_launch) ARGS;
  HGS_DISPATCH(32, 512, bwd_launch) ARGS;
#undef ARGS
  return hipErrorInvalidValue;
}

hipError_t launch_depth_normals(const float* depth, const float* T_final, const CamPack& cp, uint64_t n_pix,
                                float* normals, hipStream_t s) {
  if (n_pix == 0) return hipSuccess;
  hipLaunchKernelGGL(depth_normals_kernel, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, s, depth,
                     T_final, cp, n_pix, normals);
  return hipGetLastError();
}

}  // namespace hgs
