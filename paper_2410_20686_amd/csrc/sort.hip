// Binning of the omnidirectional rasterizer, gfx950: depth pre-sort of the (Gaussian, view)
// items, pair emission, stable LSD radix sort of the pairs by global tile, per-tile ranges.
//
// The pairs must end up ordered by the 64-bit key (global tile << 32 | depth bits), ties by
// Gaussian index.  Instead of sorting 64-bit keys over all pairs, the items (far fewer than the
// pairs) are first sorted by their 32-bit depth; pairs are then emitted in that order and sorted
// stably by tile id alone, which needs only ceil(log2(tiles) / 8) passes over the pairs.  The
// result is the same permutation as a stable sort of the 64-bit keys of index-ordered pairs.
//
// Radix sort: 8-bit digits, reduce-then-scan (no inter-workgroup spinning, so no forward-progress
// assumption): per-block digit histograms, an exclusive scan per digit across blocks, then a
// stable scatter in which each wavefront ranks its keys with 8 ballots (multi-split).
// Every count the kernels need (number of pairs) is read from device memory, so the whole
// chain runs without a host round trip and can be captured in a graph.
#include "common.h"

namespace odgs {
namespace {

__device__ inline uint32_t wave_incl_scan(uint32_t x) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

// Inclusive scan across a 256-thread block.  `lds` holds 4 words; contains two barriers.
__device__ inline uint32_t block_incl_scan256(uint32_t x, uint32_t* lds, uint32_t& total) {
  const uint32_t incl = wave_incl_scan(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  if (lane == kWave - 1) lds[w] = incl;
  __syncthreads();
  uint32_t pre = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) pre += (k < w) ? lds[k] : 0u;
  total = lds[0] + lds[1] + lds[2] + lds[3];
  __syncthreads();
  return incl + pre;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, uint32_t value, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

__device__ inline uint32_t active_count(const uint32_t* n_dev, uint32_t n_host) {
  return n_dev ? min(*n_dev, n_host) : n_host;
}

// Per-block histogram of the digit of `dbits` (<= 8) bits at `shift`: hist[digit * nblocks + block].  Each
// wavefront counts into its own LDS histogram (a quarter of the same-address atomics), reading
// four consecutive keys per 16-byte load.  AGG (for a pass over a key's top digit, which takes few
// distinct values): the lanes of a round holding the same digit are found by ballots over its
// bits and only the lowest of them adds their number, instead of one contended atomic per key.
template <bool AGG>
__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys,
                                                                 const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                                 int shift, int dbits, uint32_t* __restrict__ hist,
                                                                 int nblocks) {
  const uint32_t dmask = (1u << dbits) - 1u;
  constexpr int NW = kSortThreads / kWave;
  __shared__ uint32_t h[NW][256];
  const int t = threadIdx.x, wave = t >> 6;
  const uint32_t n = active_count(n_dev, n_host);
  const uint32_t start = blockIdx.x * (uint32_t)kSortBlockItems;
  if (start >= n) return;  // uniform: blocks past the keys are neither scanned nor scattered
#pragma unroll
  for (int w = 0; w < NW; ++w) h[w][t] = 0;
  __syncthreads();
  if constexpr (AGG) {
    const int lane = t & (kWave - 1);
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    uint32_t k[kSortIpt];
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r)  // unconditional loads stay in flight together
      k[r] = keys[min(start + (uint32_t)(r * kSortThreads + t), n - 1)];
#pragma unroll
    for (int r = 0; r < kSortIpt; ++r) {
      const uint32_t idx = start + (uint32_t)(r * kSortThreads + t);
      const bool valid = idx < n;
      const uint32_t d = (k[r] >> shift) & dmask;
      uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
      for (int b = 0; b < dbits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
        peers &= bit ? bb : ~bb;
      }
      if (valid && (peers & below) == 0ull) atomicAdd(&h[wave][d], (uint32_t)__popcll(peers));
    }
  } else if (start + (uint32_t)kSortBlockItems <= n) {  // a whole block: 16-byte loads, all in flight
    uint4 k4[kSortIpt / 4];
#pragma unroll
    for (int r = 0; r < kSortIpt / 4; ++r)
      k4[r] = *reinterpret_cast<const uint4*>(keys + start + 4u * (uint32_t)(r * kSortThreads + t));
#pragma unroll
    for (int r = 0; r < kSortIpt / 4; ++r) {
      atomicAdd(&h[wave][(k4[r].x >> shift) & dmask], 1u);
      atomicAdd(&h[wave][(k4[r].y >> shift) & dmask], 1u);
      atomicAdd(&h[wave][(k4[r].z >> shift) & dmask], 1u);
      atomicAdd(&h[wave][(k4[r].w >> shift) & dmask], 1u);
    }
  } else {
    for (uint32_t i = start + (uint32_t)t; i < n; i += kSortThreads) atomicAdd(&h[wave][(keys[i] >> shift) & dmask], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) c += h[w][t];
  hist[t * nblocks + blockIdx.x] = c;
}

// Block d: exclusive scan of hist[d][0..live) in place, over the blocks that hold keys; digit
// total to digit_tot[d].  Each thread takes kDigitIpt consecutive entries per round, so a row of
// thousands of sort blocks needs a few block-wide scans rather than one per 256 entries.
constexpr int kDigitIpt = 8;

__global__ __launch_bounds__(256) void radix_digit_scan_kernel(uint32_t* __restrict__ hist, int nblocks,
                                                               const uint32_t* __restrict__ n_dev, uint32_t n_host,
                                                               uint32_t* __restrict__ digit_tot) {
  __shared__ uint32_t lds[4];
  uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
  const uint32_t n = active_count(n_dev, n_host);
  const int live = min(nblocks, (int)((n + (uint32_t)kSortBlockItems - 1) / (uint32_t)kSortBlockItems));
  uint32_t carry = 0;
  for (int base = 0; base < live; base += 256 * kDigitIpt) {
    const int k0 = base + (int)threadIdx.x * kDigitIpt;
    uint32_t x[kDigitIpt], sum = 0;
#pragma unroll
    for (int j = 0; j < kDigitIpt; ++j) {
      x[j] = k0 + j < live ? row[k0 + j] : 0u;
      sum += x[j];
    }
    uint32_t total;
    uint32_t run = carry + block_incl_scan256(sum, lds, total) - sum;
#pragma unroll
    for (int j = 0; j < kDigitIpt; ++j) {
      if (k0 + j < live) row[k0 + j] = run;
      run += x[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

// Stable scatter of one digit pass (a digit of `dbits` <= 8 bits at `shift`).  vin == nullptr
// means the values are the input positions.
// Phase 1: each wavefront ranks its own contiguous quarter of the block's keys (rounds of 64 in
// input order; per round a multi-split by dbits ballots gives the rank among same-digit peers, added
// to the wavefront's running per-digit count in LDS) with no block barriers; one exclusive prefix
// over the wavefronts per digit then makes the ranks block-wide and stable.  Phase 2 places the
// keys digit-sorted in LDS; phase 3 writes them out in that order, so consecutive threads store
// consecutive addresses of each digit's output run.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ n_dev, uint32_t n_host, int shift, int dbits,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ digit_tot, int nblocks) {
  const uint32_t dmask = (1u << dbits) - 1u;
  constexpr int NW = kSortThreads / kWave;
  constexpr int PER_WAVE = kSortBlockItems / NW;
  constexpr int ROUNDS = PER_WAVE / kWave;
  __shared__ uint32_t s_key[kSortBlockItems];
  __shared__ uint32_t s_val[kSortBlockItems];
  __shared__ uint32_t wh[NW][256];    // per-wavefront running digit counts, then local placement starts
  __shared__ uint32_t gshift[256];    // global start minus local start of each digit for this block
  __shared__ uint32_t lds[4];
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t >> 6;
  const uint32_t n = active_count(n_dev, n_host);
  const uint32_t start = blockIdx.x * (uint32_t)kSortBlockItems;
  if (start >= n) return;  // uniform across the block
  const uint32_t nb = min((uint32_t)kSortBlockItems, n - start);
  uint32_t total;
  const uint32_t dt = digit_tot[t];
  const uint32_t incl = block_incl_scan256(dt, lds, total);
  const uint32_t gstart = incl - dt + hist[t * nblocks + blockIdx.x];  // global start of digit t
#pragma unroll
  for (int w = 0; w < NW; ++w) wh[w][t] = 0;
  __syncthreads();
  const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  uint32_t key[ROUNDS], val[ROUNDS], rank[ROUNDS];
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const uint32_t li = (uint32_t)(wave * PER_WAVE + r * kWave + lane);
    const bool valid = li < nb;
    key[r] = valid ? kin[start + li] : 0u;
    val[r] = valid ? (vin ? vin[start + li] : start + li) : 0u;
  }
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const uint32_t li = (uint32_t)(wave * PER_WAVE + r * kWave + lane);
    const bool valid = li < nb;
    const uint32_t d = (key[r] >> shift) & dmask;
    uint64_t peers = __builtin_amdgcn_ballot_w64(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b >= dbits) break;  // uniform
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t wr = __popcll(peers & lanes_below);
    // every lane of a peer group reads the group's running count, then its first lane advances it
    // (one wavefront's LDS operations execute in order)
    const uint32_t base = wh[wave][d];
    __builtin_amdgcn_wave_barrier();
    rank[r] = base + wr;
    if (valid && wr == 0) wh[wave][d] = base + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: block-local start (exclusive prefix over digits of the block totals) plus the
  // wavefront's exclusive prefix, folded into one placement start per (wavefront, digit); and
  // the digit's global-minus-local shift for the write-out (one LDS read per key in each phase)
  {
    uint32_t run = 0;
    uint32_t c[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      c[w] = wh[w][t];
      run += c[w];
    }
    const uint32_t ci = block_incl_scan256(run, lds, total);
    uint32_t start = ci - run;  // local start of digit t
    gshift[t] = gstart - start;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      wh[w][t] = start;
      start += c[w];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ROUNDS; ++r) {
    const uint32_t li = (uint32_t)(wave * PER_WAVE + r * kWave + lane);
    if (li < nb) {
      const uint32_t d = (key[r] >> shift) & dmask;
      const uint32_t p = wh[wave][d] + rank[r];
      s_key[p] = key[r];
      s_val[p] = val[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortIpt; ++r) {
    const uint32_t i = r * kSortThreads + t;
    if (i < nb) {
      const uint32_t k = s_key[i];
      const uint32_t d = (k >> shift) & dmask;
      const uint32_t pos = gshift[d] + i;  // unsigned wrap-around: global start + (i - local start)
      if (pos < n) {  // always true for a consistent histogram; keeps a corrupted one in bounds
        kout[pos] = k;
        vout[pos] = s_val[i];
      }
    }
  }
}

// Sum of the tile counts of each block of depth-sorted items.
constexpr int kScanIpt = 4;
constexpr int kScanBlockItems = 256 * kScanIpt;

// Coarse binning (16x16 tiles, every W and H a multiple of 32): an item's pairs are the 32x32
// tiles its 16x16-tile rectangle r touches, columns c0 .. c0 + nc - 1 (an unwrapped range, taken
// modulo W / 32 like r's own columns) and rows r0 .. r0 + nr - 1, each pair carrying the mask of
// the four 16x16 tiles b = 2 by + bx of its 32x32 tile that r covers.
struct CoarseRect {
  int c0, nc, r0, nr;
};

__device__ inline CoarseRect coarse_rect(const Rect& r, int ntx16) {
  CoarseRect c{0, 0, 0, 0};
  if (r.ncols == 0 || r.nrows == 0) return c;
  if (r.ncols >= ntx16) {  // every column (col0 = 0)
    c.nc = ntx16 >> 1;
  } else {
    c.c0 = r.col0 >> 1;
    c.nc = ((r.col0 + r.ncols - 1) >> 1) - c.c0 + 1;
  }
  c.r0 = r.row0 >> 1;
  c.nr = ((r.row0 + r.nrows - 1) >> 1) - c.r0 + 1;
  return c;
}

// Mask of the 16x16 tiles of 32x32 tile (column cu, unwrapped; row ru) that r covers.
__device__ inline uint32_t coarse_mask(const Rect& r, int ntx16, int cu, int ru) {
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int x = 2 * cu + (b & 1), y = 2 * ru + (b >> 1);
    const bool col = r.ncols >= ntx16 || (x >= r.col0 && x < r.col0 + r.ncols);
    const bool row = y >= r.row0 && y < r.row0 + r.nrows;
    m |= (col && row) ? (1u << b) : 0u;
  }
  return m;
}

// Key bits above the coarse tile id: the 16x16-tile mask (coarse tile ids stay below 2^27).
constexpr int kMaskShift = 28;
constexpr uint32_t kTileIdMask = (1u << kMaskShift) - 1u;

// Gathers the items' tile rectangles into depth order (the one random access of binning; the
// offset and emission passes then read them sequentially), writes each item's pair count in depth
// order (scnt; 32x32 tiles with coarse binning) and reduces the counts per block.
__global__ __launch_bounds__(256) void count_reduce_kernel(const uint32_t* __restrict__ sorted_ids,
                                                           const Rect* __restrict__ rect, int64_t items, int64_t n,
                                                           ViewTable vt, int coarse, Rect* __restrict__ srect,
                                                           uint32_t* __restrict__ scnt,
                                                           uint32_t* __restrict__ block_sum) {
  __shared__ uint32_t lds[4];
  __shared__ int s_w16[ODGS_MAX_VIEWS];  // 16x16 tiles per row of each view (coarse binning)
  if (threadIdx.x < vt.n_views) s_w16[threadIdx.x] = vt.W[threadIdx.x] / 16;
  __syncthreads();
  const int64_t start = (int64_t)blockIdx.x * kScanBlockItems;
  // all loads first (indices clamped into the list), so the four gathers are in flight together
  uint32_t id[kScanIpt];
  Rect r[kScanIpt];
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    const int64_t j = start + k * 256 + threadIdx.x;  // coalesced
    id[k] = sorted_ids[j < items ? j : items - 1];
  }
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) r[k] = rect[id[k]];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    const int64_t j = start + k * 256 + threadIdx.x;
    if (j < items) {
      srect[j] = r[k];
      uint32_t c = (uint32_t)r[k].ncols * (uint32_t)r[k].nrows;
      if (coarse) {
        const CoarseRect cr = coarse_rect(r[k], s_w16[id[k] / (uint32_t)n]);  // item ids are below 2^32
        c = (uint32_t)(cr.nc * cr.nr);
      }
      scnt[j] = c;
      s += c;
    }
  }
  uint32_t total;
  block_incl_scan256(s, lds, total);
  if (threadIdx.x == 0) block_sum[blockIdx.x] = total;
}

// Exclusive scan of the block sums (in place, as 64-bit offsets) and the pair total.
__global__ __launch_bounds__(256) void count_top_kernel(const uint32_t* __restrict__ block_sum,
                                                        uint64_t* __restrict__ block_off, int nblocks,
                                                        int64_t capacity, odgs_status* __restrict__ status) {
  constexpr int IPT = 16;  // consecutive block sums per thread and round
  __shared__ uint64_t wtot[4];
  uint64_t carry = 0;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & (kWave - 1);
  for (int base = 0; base < nblocks; base += 256 * IPT) {
    const int k0 = base + (int)threadIdx.x * IPT;
    uint32_t x[IPT];
    uint64_t sum = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      x[j] = k0 + j < nblocks ? block_sum[k0 + j] : 0u;
      sum += x[j];
    }
    uint64_t incl = sum;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint64_t y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wtot[w] = incl;
    __syncthreads();
    uint64_t pre = 0;
    for (int q = 0; q < w; ++q) pre += wtot[q];
    const uint64_t total = wtot[0] + wtot[1] + wtot[2] + wtot[3];
    __syncthreads();
    uint64_t run = carry + pre + incl - sum;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      if (k0 + j < nblocks) block_off[k0 + j] = run;
      run += x[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) {
    // a new pair list: no forward has composited it yet
    const uint32_t gen = status->bin_gen + 1u;
    status->bin_gen = gen;
    status->fwd_gen = ~gen;
    status->n_pairs = (int64_t)carry;
    const int64_t stored = (int64_t)carry < capacity ? (int64_t)carry : capacity;
    status->n_pairs_stored = (int32_t)stored;
    if ((int64_t)carry > capacity) status->flags |= ODGS_STATUS_OVERFLOW;
  }
}

// First pair position of every depth-sorted item (clamped to the capacity: items starting past
// it emit nothing).  Pairs of one item are contiguous and items follow depth order, so a later
// stable sort by tile keeps (depth, index) order inside every tile.
__global__ __launch_bounds__(256) void item_offsets_kernel(const uint32_t* __restrict__ scnt,
                                                           const uint64_t* __restrict__ block_off, int64_t items,
                                                           int64_t capacity, uint32_t* __restrict__ ioff) {
  __shared__ uint32_t lds[4];
  const int64_t start = (int64_t)blockIdx.x * kScanBlockItems;
  uint32_t cnt[kScanIpt];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    const int64_t j = start + threadIdx.x * kScanIpt + k;
    cnt[k] = j < items ? scnt[j] : 0u;
    s += cnt[k];
  }
  uint32_t total;
  const uint32_t incl = block_incl_scan256(s, lds, total);
  uint64_t off = block_off[blockIdx.x] + (incl - s);
#pragma unroll
  for (int k = 0; k < kScanIpt; ++k) {
    const int64_t j = start + threadIdx.x * kScanIpt + k;
    if (j < items) ioff[j] = (uint32_t)(off < (uint64_t)capacity ? off : (uint64_t)capacity);
    off += cnt[k];
  }
}

// Pair-parallel emission: block b writes the pairs of sort block b, [b * kSortBlockItems,
// (b + 1) * kSortBlockItems), in rounds of kEmitPairs, four consecutive pairs per thread, so
// stores are coalesced whatever the items' sizes.  Per round the block locates its items with one
// search over the item offsets, stages them in LDS, and each thread finds the item of its first
// pair by a binary search in LDS.  The block also counts the low tile digit of its pairs: the
// histogram the tile sort's first pass needs (hist[digit * nblocks + b]), so that pass does not
// read the keys once more to count them.
constexpr int kEmitRun = 4;  // consecutive pairs per thread
constexpr int kEmitPairs = 256 * kEmitRun;
constexpr int kEmitRounds = kSortBlockItems / kEmitPairs;
static_assert(kEmitRounds * kEmitPairs == kSortBlockItems, "whole rounds per sort block");

// Last index in [0, n) with a[idx] <= x, for nondecreasing a with a[0] <= x, searched by one
// whole wavefront: each round probes 64 evenly spaced entries of the interval at once and keeps
// the stretch between the last probe <= x and the next one, so about four rounds of dependent
// loads cover millions of entries (a binary search takes twenty-odd).  Uniform result.
__device__ inline int64_t wave_last_le(const uint32_t* __restrict__ a, int64_t n, uint32_t x) {
  const int lane = threadIdx.x & (kWave - 1);
  int64_t lo = 0, hi = n;  // a[lo] <= x; hi == n or a[hi] > x
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + kWave - 1) / kWave;
    const int64_t idx = lo + (int64_t)lane * step;
    const bool le = idx < hi && a[idx] <= x;  // true on a prefix of the lanes, lane 0 included
    const int k = __popcll(__builtin_amdgcn_ballot_w64(le)) - 1;
    lo += (int64_t)k * step;
    hi = min(hi, lo + step);
  }
  return lo;
}

// One round of emit_pairs_kernel: pairs [p0, p1), also counted into the wavefront's histogram.
template <bool COARSE>
__device__ inline void emit_round(const uint32_t* __restrict__ sorted_ids, const uint32_t* __restrict__ ioff,
                                  const Rect* __restrict__ srect, int64_t items, int64_t n, const ViewTable& vt,
                                  int tile, uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval, uint32_t p0,
                                  uint32_t p1, uint32_t* s_off, uint32_t* s_item, Rect* s_rect, uint32_t* s_tb,
                                  uint16_t* s_ntx, const int64_t* s_range, uint32_t* hw, uint32_t dmask,
                                  const uint32_t* s_vtb, const uint16_t* s_vntx) {
  // s_range: the items holding pairs p0 and p1 - 1
  const int64_t i0 = s_range[0];
  const int m = (int)(s_range[1] - i0 + 1);  // <= kEmitPairs: every listed item owns >= 1 pair here
  // staged with every load in flight first (indices clamped into the round's items)
  constexpr int R = kEmitPairs / 256;
  uint32_t item[R], off[R];
  Rect rc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int64_t j = i0 + min(k * 256 + (int)threadIdx.x, m - 1);
    item[k] = sorted_ids[j];
    off[k] = ioff[j];
    rc[k] = srect[j];
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int t = k * 256 + (int)threadIdx.x;
    if (t < m) {
      const uint32_t v = item[k] / (uint32_t)n;  // item ids are below 2^32
      s_off[t] = off[k];
      s_item[t] = item[k];
      s_rect[t] = rc[k];
      s_tb[t] = s_vtb[v];
      s_ntx[t] = s_vntx[v];
    }
  }
  __syncthreads();
  // each thread emits kEmitRun consecutive pairs: one search, then the rectangle is walked by
  // increments (row-major, columns wrapping at the seam), and one 16-byte store per array
  static_assert(kEmitPairs == 256 * kEmitRun && kEmitRun == 4, "four consecutive pairs per thread");
  const uint32_t q = p0 + (uint32_t)(kEmitRun * threadIdx.x);
  if (q >= p1) return;
  int lo = 0, hi = m;  // largest idx with s_off[idx] <= q
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_off[mid] <= q) lo = mid;
    else hi = mid;
  }
  Rect rr = s_rect[lo];
  uint32_t ntx = s_ntx[lo];
  // the rectangle walked: the item's 16x16 tiles, or the 32x32 tiles they fall in
  CoarseRect cr{(int)rr.col0, (int)rr.ncols, (int)rr.row0, (int)rr.nrows};
  if constexpr (COARSE) cr = coarse_rect(rr, (int)ntx);
  uint32_t local = q - s_off[lo];
  uint32_t r = local / (uint32_t)cr.nc, c = local - r * (uint32_t)cr.nc;
  uint32_t key[kEmitRun], val[kEmitRun];
#pragma unroll
  for (int j = 0; j < kEmitRun; ++j) {
    const uint32_t pj = q + (uint32_t)j;
    // next item once this one's pairs are used up (items without pairs here are skipped)
    while (lo + 1 < m && s_off[lo + 1] <= pj) {
      ++lo;
      rr = s_rect[lo];
      ntx = s_ntx[lo];
      cr = CoarseRect{(int)rr.col0, (int)rr.ncols, (int)rr.row0, (int)rr.nrows};
      if constexpr (COARSE) cr = coarse_rect(rr, (int)ntx);
      r = 0;
      c = 0;
    }
    const uint32_t cu = (uint32_t)cr.c0 + c;  // unwrapped column
    if constexpr (COARSE) {
      const uint32_t ntx32 = ntx >> 1;
      const uint32_t col = cu >= ntx32 ? cu - ntx32 : cu;
      key[j] = (s_tb[lo] + (uint32_t)(cr.r0 + (int)r) * ntx32 + col) |
               (coarse_mask(rr, (int)ntx, (int)cu, cr.r0 + (int)r) << kMaskShift);
    } else {
      const uint32_t col = cu >= ntx ? cu - ntx : cu;
      key[j] = s_tb[lo] + (uint32_t)(cr.r0 + (int)r) * ntx + col;
    }
    val[j] = s_item[lo];
    if (++c == (uint32_t)cr.nc) {
      c = 0;
      ++r;
    }
  }
#pragma unroll
  for (int j = 0; j < kEmitRun; ++j)
    if (q + (uint32_t)j < p1) atomicAdd(&hw[key[j] & dmask], 1u);
  if (q + kEmitRun <= p1) {
    *reinterpret_cast<uint4*>(pkey + q) = make_uint4(key[0], key[1], key[2], key[3]);
    *reinterpret_cast<uint4*>(pval + q) = make_uint4(val[0], val[1], val[2], val[3]);
  } else {
    for (int j = 0; j < kEmitRun && q + (uint32_t)j < p1; ++j) {
      pkey[q + j] = key[j];
      pval[q + j] = val[j];
    }
  }
}

template <bool COARSE>
__global__ __launch_bounds__(256) void emit_pairs_kernel(const uint32_t* __restrict__ sorted_ids,
                                                         const uint32_t* __restrict__ ioff,
                                                         const Rect* __restrict__ srect,
                                                         const odgs_status* __restrict__ status, int64_t items,
                                                         int64_t n, ViewTable vt, int tile, uint32_t* __restrict__ pkey,
                                                         uint32_t* __restrict__ pval, uint32_t* __restrict__ hist,
                                                         int nblocks, uint32_t dmask) {
  __shared__ uint32_t s_off[kEmitPairs + 1];
  __shared__ uint32_t s_item[kEmitPairs + 1];
  __shared__ Rect s_rect[kEmitPairs + 1];
  __shared__ uint32_t s_tb[kEmitPairs + 1];
  __shared__ uint16_t s_ntx[kEmitPairs + 1];
  __shared__ int64_t s_range[kEmitRounds][2];
  __shared__ uint32_t h[kSortThreads / kWave][256];  // per-wavefront digit counts
  __shared__ uint32_t s_vtb[ODGS_MAX_VIEWS];  // per view: first global tile id (32x32 with coarse binning)
  __shared__ uint16_t s_vntx[ODGS_MAX_VIEWS];  // per view: tiles per row (16x16 with coarse binning)
  const int t = threadIdx.x;
#pragma unroll
  for (int w = 0; w < kSortThreads / kWave; ++w) h[w][t] = 0;
  if (t < vt.n_views) {
    s_vtb[t] = (uint32_t)(COARSE ? vt.tile_base32[t] : vt.tile_base[t]);
    s_vntx[t] = (uint16_t)(vt.W[t] / tile);
  }
  const uint32_t np = (uint32_t)status->n_pairs_stored;
  const uint32_t b0 = blockIdx.x * (uint32_t)kSortBlockItems;
  {
    // wavefront w finds the items holding the first and last pair of round w (all rounds' searches
    // at once: their dependent loads overlap)
    static_assert(kEmitRounds == kSortThreads / kWave, "one wavefront per round");
    const int w = t >> 6;
    const uint32_t p0 = b0 + (uint32_t)(w * kEmitPairs);
    if (p0 < np) {
      const uint32_t p1 = min(p0 + (uint32_t)kEmitPairs, np);
      const int64_t first = wave_last_le(ioff, items, p0);
      const int64_t last = wave_last_le(ioff, items, p1 - 1);
      if ((t & (kWave - 1)) == 0) {
        s_range[w][0] = first;
        s_range[w][1] = last;
      }
    }
  }
  for (int round = 0; round < kEmitRounds; ++round) {
    const uint32_t p0 = b0 + (uint32_t)(round * kEmitPairs);
    if (p0 >= np) break;  // uniform
    __syncthreads();  // the searches are done, the previous round's staging has been read
    emit_round<COARSE>(sorted_ids, ioff, srect, items, n, vt, tile, pkey, pval, p0,
                       min(p0 + (uint32_t)kEmitPairs, np), s_off, s_item, s_rect, s_tb, s_ntx, s_range[round],
                       h[t >> 6], dmask, s_vtb, s_vntx);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kSortThreads / kWave; ++w) c += h[w][t];
  hist[t * nblocks + blockIdx.x] = c;  // every (digit, block) entry, zero past the pairs
}

// Tile ranges from the sorted keys: each thread scans eight consecutive keys (two 16-byte loads
// when the run is whole) and marks where a tile's run starts and ends.
constexpr int kRangeKeys = 8;

__global__ __launch_bounds__(256) void ranges_kernel(const uint32_t* __restrict__ keys,
                                                     const odgs_status* __restrict__ status, uint2* __restrict__ ranges) {
  const uint32_t n = (uint32_t)status->n_pairs_stored;
  const uint32_t j0 = (blockIdx.x * 256 + threadIdx.x) * (uint32_t)kRangeKeys;
  if (j0 >= n) return;
  uint32_t k[kRangeKeys];
  if (j0 + kRangeKeys <= n) {
    const uint4 a = *reinterpret_cast<const uint4*>(keys + j0);
    const uint4 b = *reinterpret_cast<const uint4*>(keys + j0 + 4);
    k[0] = a.x; k[1] = a.y; k[2] = a.z; k[3] = a.w;
    k[4] = b.x; k[5] = b.y; k[6] = b.z; k[7] = b.w;
  } else {
#pragma unroll
    for (int i = 0; i < kRangeKeys; ++i) k[i] = j0 + i < n ? keys[j0 + i] : 0u;
  }
  uint32_t prev = j0 > 0 ? keys[j0 - 1] : ~k[0];
  const uint32_t after = j0 + kRangeKeys < n ? keys[j0 + kRangeKeys] : 0u;
#pragma unroll
  for (int i = 0; i < kRangeKeys; ++i) {
    const uint32_t j = j0 + i;
    if (j < n) {
      if (prev != k[i]) ranges[k[i]].x = j;
      const bool last = j + 1 == n;
      const uint32_t next = i + 1 < kRangeKeys ? k[i + 1] : after;
      if (last || next != k[i]) ranges[k[i]].y = j + 1;
    }
    prev = k[i];
  }
}

// Refinement of the coarse lists (coarse binning): the sorted 32x32-tile list is split into the
// lists of the 16x16 tiles by the masks its keys carry.  The refined list has four regions, one per
// quadrant b of a 32x32 tile (b = 2*row + column): region b holds, in list order, every pair whose
// mask has bit b, so each 16x16 tile's list is one contiguous run in (depth, index) order.  A pair's
// position is the region's base plus the number of earlier pairs with bit b: four bit counts
// scanned over the whole list, chunk by chunk (the sort's blocks), with no per-tile work.  A chunk
// is four wavefronts of kRefineIters rounds of 64 consecutive pairs.
constexpr int kRefineWavePairs = kSortBlockItems / (kSortThreads / kWave);
constexpr int kRefineIters = kRefineWavePairs / kWave;

__device__ inline void coarse_tile_of(const ViewTable& vt, int T, int& v, int& cx, int& cy) {
  v = 0;
  while (T >= vt.tile_base32[v + 1]) ++v;
  const int ntx32 = vt.W[v] / 32, lt = T - vt.tile_base32[v];
  cx = lt % ntx32;
  cy = lt / ntx32;
}

// Per-chunk counts of the four mask bits.
__global__ __launch_bounds__(kSortThreads) void refine_count_kernel(const uint32_t* __restrict__ keys,
                                                                    const odgs_status* __restrict__ status,
                                                                    uint4* __restrict__ cnt) {
  __shared__ uint32_t wc[kSortThreads / kWave][4];
  const uint32_t n = (uint32_t)status->n_pairs_stored;
  const uint32_t base = blockIdx.x * (uint32_t)kSortBlockItems;
  if (base >= n) return;  // uniform per block
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const uint32_t wbase = base + (uint32_t)(w * kRefineWavePairs) + (uint32_t)lane;
  uint32_t c[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < kRefineIters; ++i) {
    const uint32_t j = wbase + (uint32_t)(i * kWave);
    const uint32_t kj = keys[min(j, n - 1)];  // unconditional loads stay in flight together
    const uint32_t m = j < n ? kj >> kMaskShift : 0u;
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64((m >> b) & 1u));
  }
  if (lane == 0) {
#pragma unroll
    for (int b = 0; b < 4; ++b) wc[w][b] = c[b];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kSortThreads / kWave; ++q) s += wc[q][threadIdx.x];
    reinterpret_cast<uint32_t*>(cnt + blockIdx.x)[threadIdx.x] = s;
  }
}

// Exclusive scan of the chunk counts in place (one workgroup), the region bases and the coarse pair
// count into `meta` (words 0..3 and 4), and the refined pair total into the status record (the
// pair count and stored count of the 16x16 lists; overflow past the capacity as for the lists
// themselves).  When the coarse list itself overflowed, the refined count is of a truncated list:
// the pair count reported is then four times the coarse one, an upper bound of the true count (a
// coarse pair holds at most four 16x16 pairs).
__global__ __launch_bounds__(1024) void refine_scan_kernel(uint4* __restrict__ cnt, uint32_t* __restrict__ meta,
                                                           int64_t capacity, odgs_status* __restrict__ status) {
  __shared__ uint32_t wsum[1024 / kWave][4];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t >> 6;
  const uint32_t n = (uint32_t)status->n_pairs_stored;
  const int chunks = (int)((n + (uint32_t)kSortBlockItems - 1) / (uint32_t)kSortBlockItems);
  constexpr int IPT = 4;                 // consecutive chunks per thread and round
  uint32_t carry[4] = {0u, 0u, 0u, 0u};  // each bit count is at most n < 2^31
  for (int base = 0; base < chunks; base += 1024 * IPT) {
    const int k0 = base + t * IPT;
    uint4 x[IPT];
    uint32_t s[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      x[j] = k0 + j < chunks ? cnt[k0 + j] : make_uint4(0u, 0u, 0u, 0u);
      s[0] += x[j].x;
      s[1] += x[j].y;
      s[2] += x[j].z;
      s[3] += x[j].w;
    }
    uint32_t incl[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      incl[b] = wave_incl_scan(s[b]);
      if (lane == kWave - 1) wsum[w][b] = incl[b];
    }
    __syncthreads();
    uint32_t ex[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t pre = 0, total = 0;
      for (int q = 0; q < 1024 / kWave; ++q) {
        pre += q < w ? wsum[q][b] : 0u;
        total += wsum[q][b];
      }
      ex[b] = carry[b] + pre + incl[b] - s[b];
      carry[b] += total;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
      if (k0 + j < chunks) cnt[k0 + j] = make_uint4(ex[0], ex[1], ex[2], ex[3]);
      ex[0] += x[j].x;
      ex[1] += x[j].y;
      ex[2] += x[j].z;
      ex[3] += x[j].w;
    }
  }
  __syncthreads();  // every thread has read the stored count
  if (t == 0) {
    int64_t r = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      meta[b] = (uint32_t)(r < capacity ? r : capacity);
      r += carry[b];
    }
    meta[4] = n;
    const bool truncated = (status->flags & ODGS_STATUS_OVERFLOW) != 0;
    status->n_pairs = truncated ? 4 * status->n_pairs : r;
    status->n_pairs_stored = (int32_t)(r < capacity ? r : capacity);
    if (r > capacity) status->flags |= ODGS_STATUS_OVERFLOW;
  }
}

// The writes: each wavefront recounts its pairs' bits before each round of 64 (ballots), so the
// pairs of one region that a round holds land in consecutive positions.  The pair that starts a
// 32x32 tile's run sets the starts of its four 16x16 tiles' ranges, the one that ends it the ends.
__global__ __launch_bounds__(kSortThreads) void refine_write_kernel(
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, const uint4* __restrict__ pre,
    const uint32_t* __restrict__ meta, ViewTable vt, uint32_t capacity, uint32_t* __restrict__ out,
    uint2* __restrict__ ranges16) {
  __shared__ uint32_t wc[kSortThreads / kWave][4];
  const uint32_t n = meta[4];
  const uint32_t base = blockIdx.x * (uint32_t)kSortBlockItems;
  if (base >= n) return;  // uniform per block
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  const uint32_t wbase = base + (uint32_t)(w * kRefineWavePairs);
  uint32_t key[kRefineIters], val[kRefineIters];
  uint32_t c[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int i = 0; i < kRefineIters; ++i) {
    const uint32_t j = wbase + (uint32_t)(i * kWave + lane);
    const uint32_t jc = min(j, n - 1);  // unconditional loads stay in flight together
    key[i] = keys[jc];
    val[i] = vals[jc];
    if (j >= n) key[i] = 0u;  // no mask bits past the list
    const uint32_t m = key[i] >> kMaskShift;
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64((m >> b) & 1u));
  }
  if (lane == 0) {
#pragma unroll
    for (int b = 0; b < 4; ++b) wc[w][b] = c[b];
  }
  __syncthreads();
  const uint4 p4 = pre[blockIdx.x];
  uint32_t run[4] = {meta[0] + p4.x, meta[1] + p4.y, meta[2] + p4.z, meta[3] + p4.w};
  for (int q = 0; q < w; ++q) {
#pragma unroll
    for (int b = 0; b < 4; ++b) run[b] += wc[q][b];
  }
  // tile of the pair before this lane's first one
  uint32_t last = wbase > 0 && wbase - 1 < n ? keys[wbase - 1] & kTileIdMask : 0xFFFFFFFFu;
#pragma unroll
  for (int i = 0; i < kRefineIters; ++i) {
    const uint32_t j = wbase + (uint32_t)(i * kWave + lane);
    const bool live = j < n;
    const uint32_t m = key[i] >> kMaskShift, t = key[i] & kTileIdMask;
    const uint32_t up = __shfl_up(t, 1);
    const uint32_t prev = lane == 0 ? last : up;
    // tile of the pair after this one (lane 63: the next round's first pair); none past the list
    const uint32_t down = __shfl_down(t, 1);
    const uint32_t first = i + 1 < kRefineIters ? __shfl(key[i + 1], 0) & kTileIdMask : 0u;
    uint32_t next = down;
    if (lane == kWave - 1)
      next = i + 1 < kRefineIters ? first : (j + 1 < n ? keys[j + 1] & kTileIdMask : 0xFFFFFFFFu);
    if (j + 1 >= n) next = 0xFFFFFFFFu;
    last = __shfl(t, kWave - 1);
    uint32_t g[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t bit = (m >> b) & 1u;
      const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
      g[b] = run[b] + (uint32_t)__popcll(bb & below);
      if (bit && g[b] < capacity) out[g[b]] = val[i];
      run[b] += (uint32_t)__popcll(bb);
    }
    const bool head = live && prev != t, tail = live && next != t;
    if (head || tail) {
      int v, cx, cy;
      coarse_tile_of(vt, (int)t, v, cx, cy);
      const int ntx16 = vt.W[v] / 16;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int tile16 = vt.tile_base[v] + (2 * cy + (b >> 1)) * ntx16 + 2 * cx + (b & 1);
        if (head) ranges16[tile16].x = min(g[b], capacity);
        if (tail) ranges16[tile16].y = min(g[b] + ((m >> b) & 1u), capacity);
      }
    }
  }
}

// Work queue of the compositors: every global tile id, in descending order of its list length
// (the tile's compositing cost), bucketed on a logarithmic scale with 32 buckets per octave (the
// order inside a bucket is arbitrary).  Three small launches: per-block bucket counts, one scan
// that turns them into per-(block, bucket) starts, and the scatter.
constexpr int kQueueBuckets = 1024;
constexpr int kQueueTiles = 4096;  // tiles per block of the count and scatter kernels (16 per thread)
// A list is split into quadrant tasks (for compositors that take them) when one wavefront alone
// would take long against the whole launch: when it holds at least 1 / kSplitShare of all pairs
// and, with kSplitAllTiles tiles or more, at least kSplitLen pairs (with fewer tiles than that the
// device has wavefront slots to spare, and every list is split).  At most split_tile_cap(tiles)
// lists are split: an eighth of the tiles, or kSplitCapMin.
constexpr uint32_t kSplitLen = 1024;
constexpr uint32_t kSplitShare = 4096;
constexpr int kSplitAllTiles = 4096;
constexpr int kSplitCapMin = 1024;

__device__ inline uint32_t cost_bucket(uint32_t len) {
  // 0 for an empty list, else 1 + 32 log2(len) (exponent and top five mantissa bits; <= 993)
  return len == 0 ? 0u : 1u + ((__float_as_uint((float)len) - 0x3f800000u) >> 18);
}

// bstart[block][bucket] = number of the block's tiles in the bucket (every entry written).
__global__ __launch_bounds__(256) void queue_count_kernel(const uint2* __restrict__ ranges, int tiles,
                                                          uint32_t* __restrict__ bstart) {
  __shared__ uint32_t h[kQueueBuckets];
  for (int b = threadIdx.x; b < kQueueBuckets; b += 256) h[b] = 0;
  __syncthreads();
  for (int k = 0; k < kQueueTiles / 256; ++k) {
    const int i = blockIdx.x * kQueueTiles + k * 256 + threadIdx.x;
    if (i < tiles) {
      const uint2 r = ranges[i];
      atomicAdd(&h[cost_bucket(r.y - r.x)], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kQueueBuckets; b += 256) bstart[(size_t)blockIdx.x * kQueueBuckets + b] = h[b];
}

// Buckets in descending order, blocks in order: the counts become each (block, bucket)'s first
// queue position.  One workgroup; also clears the persistent launches' counters and records the
// number of tiles to split (those with lists of kSplitLen or more, at most split_cap).
__global__ __launch_bounds__(kQueueBuckets) void queue_scan_kernel(uint32_t* __restrict__ bstart, int nblocks,
                                                                   uint32_t* __restrict__ ctr, uint32_t split_cap,
                                                                   uint32_t split_floor,
                                                                   const uint32_t* __restrict__ n_pairs) {
  __shared__ uint32_t wsum[kQueueBuckets / kWave];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t >> 6;
  const int bucket = kQueueBuckets - 1 - t;
  if (t < 4) ctr[t] = 0u;
  uint32_t c = 0;
  for (int b = 0; b < nblocks; ++b) c += bstart[(size_t)b * kQueueBuckets + bucket];
  const uint32_t incl = wave_incl_scan(c);
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - c;
  for (int k = 0; k < w; ++k) run += wsum[k];
  // tiles in this bucket or above: the first run + c queue entries
  if (bucket == (int)cost_bucket(max(split_floor, *n_pairs / kSplitShare))) ctr[4] = min(run + c, split_cap);
  for (int b = 0; b < nblocks; ++b) {
    uint32_t* e = bstart + (size_t)b * kQueueBuckets + bucket;
    const uint32_t x = *e;
    *e = run;
    run += x;
  }
}

__global__ __launch_bounds__(256) void queue_scatter_kernel(const uint2* __restrict__ ranges, int tiles,
                                                            const uint32_t* __restrict__ bstart,
                                                            uint32_t* __restrict__ order) {
  __shared__ uint32_t cur[kQueueBuckets];
  for (int b = threadIdx.x; b < kQueueBuckets; b += 256) cur[b] = bstart[(size_t)blockIdx.x * kQueueBuckets + b];
  __syncthreads();
  for (int k = 0; k < kQueueTiles / 256; ++k) {
    const int i = blockIdx.x * kQueueTiles + k * 256 + threadIdx.x;
    if (i < tiles) {
      const uint2 r = ranges[i];
      order[atomicAdd(&cur[cost_bucket(r.y - r.x)], 1u)] = (uint32_t)i;
    }
  }
}

hipError_t launch_tile_queue(const uint2* ranges, int tiles, const uint32_t* n_pairs, uint32_t* bstart,
                             uint32_t* queue, hipStream_t st) {
  const int nb = (tiles + kQueueTiles - 1) / kQueueTiles;
  if (nb > 0) hipLaunchKernelGGL(queue_count_kernel, dim3(nb), dim3(256), 0, st, ranges, tiles, bstart);
  hipLaunchKernelGGL(queue_scan_kernel, dim3(1), dim3(kQueueBuckets), 0, st, bstart, nb, queue,
                     (uint32_t)split_tile_cap(tiles), tiles >= kSplitAllTiles ? kSplitLen : 1u, n_pairs);
  if (nb > 0) hipLaunchKernelGGL(queue_scatter_kernel, dim3(nb), dim3(256), 0, st, ranges, tiles, bstart, queue + 16);
  return hipGetLastError();
}

__global__ void status_reset_kernel(odgs_status* st) {
  if (threadIdx.x == 0) {
    st->flags = 0;
    st->n_pairs_stored = 0;
    st->n_pairs = 0;
    st->n_visible = 0;
    st->n_culled = 0;
    st->n_nonfinite = 0;
    st->fwd_gen = ~st->bin_gen;  // bin_gen survives resets
  }
}

// Digit width of each pass over `bits` key bits: as many passes as 8-bit digits would take, the
// bits spread evenly over them (14 bits: two 7-bit passes, whose scatters write runs twice as long
// as an 8-bit digit's).
int sort_digit_bits(int bits) {
  const int passes = (bits + 7) / 8;
  return (bits + passes - 1) / passes;
}

// first_hist: the first pass's histogram is already in `hist` (written by the producer of the keys).
hipError_t radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, bool identity_vals,
                      const uint32_t* n_dev, uint32_t n_host, int bits, int nblocks, uint32_t* hist,
                      uint32_t* digit_tot, hipStream_t st, bool first_hist = false) {
  uint32_t* kb[2] = {k0, k1};
  uint32_t* vb[2] = {v0, v1};
  int cur = 0;
  const int dw = sort_digit_bits(bits);
  for (int shift = 0; shift < bits; shift += dw) {
    const uint32_t* vin = (shift == 0 && identity_vals) ? nullptr : vb[cur];
    const int dbits = bits - shift < dw ? bits - shift : dw;
    if (shift > 0 || !first_hist) {
      if (shift + dw >= bits)  // the top digit: few distinct values
        hipLaunchKernelGGL(radix_hist_kernel<true>, dim3(nblocks), dim3(kSortThreads), 0, st, kb[cur], n_dev, n_host,
                           shift, dbits, hist, nblocks);
      else
        hipLaunchKernelGGL(radix_hist_kernel<false>, dim3(nblocks), dim3(kSortThreads), 0, st, kb[cur], n_dev, n_host,
                           shift, dbits, hist, nblocks);
    }
    hipLaunchKernelGGL(radix_digit_scan_kernel, dim3(256), dim3(256), 0, st, hist, nblocks, n_dev, n_host, digit_tot);
    hipLaunchKernelGGL(radix_scatter_kernel, dim3(nblocks), dim3(kSortThreads), 0, st, kb[cur], vin, kb[cur ^ 1],
                       vb[cur ^ 1], n_dev, n_host, shift, dbits, hist, digit_tot, nblocks);
    cur ^= 1;
  }
  return hipGetLastError();
}

}  // namespace

int sort_passes(int bits) { return (bits + 7) / 8; }

hipError_t launch_status_reset(const odgs_plan* p, void* ws, hipStream_t st) {
  hipLaunchKernelGGL(status_reset_kernel, dim3(1), dim3(64), 0, st, ws_ptr<odgs_status>(ws, p->off_status));
  return hipGetLastError();
}

TileSched make_sched(const odgs_plan* p, void* ws, int which) {
  uint32_t* q = ws_ptr<uint32_t>(ws, p->off_queue);
  TileSched s{};
  s.status = ws_ptr<odgs_status>(ws, p->off_status);
  s.tiles = p->tile_base[p->n_views];
  s.order = (p->s.flags & ODGS_FLAG_SCHED_TILE_ID) ? nullptr : q + 16;  // after 64 bytes of counters
  s.ctr = (p->s.flags & ODGS_FLAG_SCHED_PERSISTENT) ? q + 2 * which : nullptr;
  s.split = q + 4;
  s.split_cap = 0;
  s.split_all = 0;
  return s;
}

int split_tile_cap(int tiles) { return tiles < kSplitCapMin ? tiles : std::max(kSplitCapMin, tiles / 8); }

int sched_grid(const TileSched& s, int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 1;
  const int64_t g = (int64_t)cus * (per_cu > 0 ? per_cu : 1);
  return (int)(g < sched_tasks(s) ? g : sched_tasks(s));
}

hipError_t launch_fill_u32(uint32_t* ptr, uint32_t value, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, ptr, value, n);
  return hipGetLastError();
}

hipError_t launch_bin_sort(const odgs_plan* p, void* ws, hipStream_t st) {
  odgs_status* status = ws_ptr<odgs_status>(ws, p->off_status);
  const int64_t items = p->items;
  uint32_t* hist = ws_ptr<uint32_t>(ws, p->off_hist);
  uint32_t* digit = ws_ptr<uint32_t>(ws, p->off_digit);
  uint2* ranges = ws_ptr<uint2>(ws, p->off_ranges);
  hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2 * (int64_t)p->tile_base[p->n_views], st);
  if (e != hipSuccess) return e;
  const int tiles = p->tile_base[p->n_views];
  uint32_t* queue = ws_ptr<uint32_t>(ws, p->off_queue);
  const uint32_t* n_dev = reinterpret_cast<const uint32_t*>(&status->n_pairs_stored);
  if (items == 0) return launch_tile_queue(ranges, tiles, n_dev, hist, queue, st);
  // 1. items by radial depth (culled items carry the largest key)
  uint32_t* dk[2] = {ws_ptr<uint32_t>(ws, p->off_dkey[0]), ws_ptr<uint32_t>(ws, p->off_dkey[1])};
  uint32_t* di[2] = {ws_ptr<uint32_t>(ws, p->off_did[0]), ws_ptr<uint32_t>(ws, p->off_did[1])};
  e = radix_sort(dk[0], di[0], dk[1], di[1], true, nullptr, (uint32_t)items, 32, p->item_blocks, hist, digit, st);
  if (e != hipSuccess) return e;
  const uint32_t* sorted_ids = di[p->depth_final];
  // 2. pair offsets in depth order, and P
  const int sblocks = (int)((items + kScanBlockItems - 1) / kScanBlockItems);
  uint32_t* bsum = ws_ptr<uint32_t>(ws, p->off_blocksum);
  uint64_t* boff = reinterpret_cast<uint64_t*>(bsum + align_up((size_t)sblocks, 64));
  Rect* srect = ws_ptr<Rect>(ws, p->off_srect);
  const ViewTable vt = make_view_table(p);
  const bool coarse = p->coarse != 0;
  uint32_t* scnt = di[p->depth_final ^ 1];  // per-item pair counts in depth order (free id buffer)
  hipLaunchKernelGGL(count_reduce_kernel, dim3(sblocks), dim3(256), 0, st, sorted_ids, ws_ptr<Rect>(ws, p->off_rect),
                     items, p->n, vt, coarse ? 1 : 0, srect, scnt, bsum);
  hipLaunchKernelGGL(count_top_kernel, dim3(1), dim3(256), 0, st, bsum, boff, sblocks, p->pair_capacity, status);
  // 3. emit pairs: per-item offsets (into the free ping-pong buffer), then pair-parallel writes
  uint32_t* pk[2] = {ws_ptr<uint32_t>(ws, p->off_pkey[0]), ws_ptr<uint32_t>(ws, p->off_pkey[1])};
  uint32_t* pv[2] = {ws_ptr<uint32_t>(ws, p->off_pval[0]), ws_ptr<uint32_t>(ws, p->off_pval[1])};
  uint32_t* ioff = dk[p->depth_final ^ 1];
  hipLaunchKernelGGL(item_offsets_kernel, dim3(sblocks), dim3(256), 0, st, scnt, boff, items, p->pair_capacity,
                     ioff);
  const int bits = coarse ? p->coarse_bits : p->tile_bits;
  const uint32_t dmask0 = (1u << sort_digit_bits(bits)) - 1u;  // the first tile pass's digit
  if (p->pair_blocks > 0) {
    if (coarse)
      hipLaunchKernelGGL(emit_pairs_kernel<true>, dim3((unsigned)p->pair_blocks), dim3(kSortThreads), 0, st,
                         sorted_ids, ioff, srect, status, items, p->n, vt, p->s.tile, pk[0], pv[0], hist,
                         p->pair_blocks, dmask0);
    else
      hipLaunchKernelGGL(emit_pairs_kernel<false>, dim3((unsigned)p->pair_blocks), dim3(kSortThreads), 0, st,
                         sorted_ids, ioff, srect, status, items, p->n, vt, p->s.tile, pk[0], pv[0], hist,
                         p->pair_blocks, dmask0);
  }
  // 4. stable sort of the pairs by global tile (the first pass's histogram counted by the emission)
  e = radix_sort(pk[0], pv[0], pk[1], pv[1], false, n_dev, (uint32_t)p->pair_capacity, bits, p->pair_blocks, hist,
                 digit, st, true);
  if (e != hipSuccess) return e;
  const int sorted = sort_passes(bits) % 2;  // the buffer pair holding the sorted list
  if (!coarse) {
    // 5. tile ranges
    hipLaunchKernelGGL(ranges_kernel, dim3((unsigned)((p->pair_capacity + 256 * kRangeKeys - 1) / (256 * kRangeKeys))),
                       dim3(256), 0, st, pk[sorted], status, ranges);
  } else {
    // 5. the 32x32 tiles' list split into the 16x16 tiles' lists and ranges, in the other pair
    //    buffer (scratch: the free radix histograms)
    uint4* cnt = reinterpret_cast<uint4*>(hist);  // per chunk (sort block)
    uint32_t* meta = hist + align_up((size_t)p->pair_blocks * 4, 64);
    const unsigned cgrid = (unsigned)p->pair_blocks;
    hipLaunchKernelGGL(refine_count_kernel, dim3(cgrid), dim3(kSortThreads), 0, st, pk[sorted], status, cnt);
    hipLaunchKernelGGL(refine_scan_kernel, dim3(1), dim3(1024), 0, st, cnt, meta, p->pair_capacity, status);
    hipLaunchKernelGGL(refine_write_kernel, dim3(cgrid), dim3(kSortThreads), 0, st, pk[sorted], pv[sorted], cnt, meta,
                       vt, (uint32_t)p->pair_capacity, pv[sorted ^ 1], ranges);
  }
  // 6. the compositors' work queue, longest list first (its scratch: the free radix histograms)
  return launch_tile_queue(ranges, tiles, n_dev, hist, queue, st);
}

}  // namespace odgs
