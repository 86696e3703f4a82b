// Compositing kernels of the omnidirectional rasterizer, gfx950.
//
// Pixels are grouped in 8x8 quadrants.  At tiles of 16 and 32 one 64-wide wavefront composites a
// 16x16 block, four pixels per lane (lane l holds pixel (l % 8, l / 8) of each quadrant): a whole
// 16x16 tile, one quadrant of a split tile, or one of the four blocks of a 32x32 tile (the tasks
// of TileSched).  At tiles of 8, and in the counting and depth variants of the forward, one
// workgroup per (view, tile) with one pixel per lane, each wavefront owning one quadrant.  The
// tile's depth-ordered list is staged through LDS in batches; while the forward stages, each
// record gets a bit mask of the quadrants its footprint can reach, so a quadrant skips, with a
// uniform branch, every Gaussian that cannot reach any of its pixels.  (The mask is conservative: a
// skipped Gaussian has alpha < 1/255 at every pixel of the quadrant, so results are identical to
// testing every pixel.)  The forward stores the masks per list position and the backward loads
// them.
//
// Forward: front-to-back compositing (Eq. gaussian2d, Eq. alphablending) until a pixel's
// transmittance would drop below 1e-4; the workgroup stops loading batches once every pixel is
// done.  Backward: back to front from the last contributor, transmittance recovered by
// multiplying with 1/(1 - alpha); the nine per-pixel gradients of the 2D quantities are summed
// over each 16-lane row by a DPP butterfly that leaves one value per lane, over the four rows by
// the row-swap permutes, kept per wavefront in LDS, and reach global memory with one double atomic
// per (Gaussian, tile, quantity), so the totals do not depend on the order in which tiles finish.
// One launch covers all views of a step: the grid spans the global tile ids of every view.
#include <type_traits>
#include <utility>

#include "common.h"
#include "wave.h"

namespace odgs {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;

template <int CTRL, int ROW_MASK>
__device__ inline float dpp_shift_add(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
  return v + __int_as_float(s);
}

// Wavefront sum by DPP; the total lands in lane 63.
__device__ inline float wave_sum_to_lane63(float v) {
  v = dpp_shift_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]: pairs
  v = dpp_shift_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]: quads
  v = dpp_shift_add<0x141, 0xF>(v);  // row_half_mirror: 8 lanes
  v = dpp_shift_add<0x140, 0xF>(v);  // row_mirror: 16-lane rows
  v = dpp_shift_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_shift_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

__device__ inline float lane63(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }


// Sums nine per-lane values over each 16-lane row in four DPP exchange steps (pairs (i, 15-i),
// (i, 7-i), (i, 3-i), (i, i^1) inside the row).  Values 0..7 are transposed (each step halves the
// slots a lane holds: value index = lane bits 3,2,1 read as 4*b3 + 2*b2 + b1 on even lanes); value
// 8 is summed in place through the first three steps and takes the odd lanes in the last one.
// Lane i ends with the row sum of value kRowSlot[i % 16] (none where the table says 15; value 8,
// held by all eight odd lanes, is assigned to lane 1 only).
constexpr uint64_t kRowSlot = 0xF7F6F5F4F3F2F180ull;  // nibble i = value index held by row lane i


// Sum of a value over the eight lanes of an aligned 8-lane group (every lane gets the sum).
__device__ inline float group8_sum(float x) {
  x += dpp_read<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_read<0x4E>(x);   // quad_perm [2,3,0,1]
  return x + dpp_read<0x141>(x);  // row_half_mirror: the other quad of the 8-lane group
}

// Wavefront sum of one value, in every lane.
__device__ inline float wave_sum(float x) {
  x = group8_sum(x);
  x += dpp_read<0x140>(x);  // row_mirror: the other half of the 16-lane row
  return sum_rows(x);
}

// Nine per-lane values summed over the wavefront with most of the data movement in LDS.
// Values 0..7 go value-major into the wavefront's scratch red[8][kRedStride]; lane 8j+m later
// reads entries 8m..8m+7 of value j, adds them, and an 8-lane DPP sum completes the total
// (held by lane 8j).  The reads are issued one accepted entry later, so their latency overlaps
// that entry's arithmetic; value 8 is summed with DPP directly.  LDS executes one wavefront's
// operations in order, so only compiler reordering across the wave barriers must be prevented.
constexpr int kRedStride = 68;  // padded rows (16-byte aligned)

__device__ inline void red_write(float (&red)[8][kRedStride], const float (&g)[9], int lane) {
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int q = 0; q < 8; ++q) red[q][lane] = g[q];
  __builtin_amdgcn_wave_barrier();
}

__device__ inline void red_read(const float (&red)[8][kRedStride], int lane, float4& r0, float4& r1) {
  __builtin_amdgcn_wave_barrier();
  const int j = lane >> 3, m = lane & 7;
  r0 = *reinterpret_cast<const float4*>(&red[j][8 * m]);
  r1 = *reinterpret_cast<const float4*>(&red[j][8 * m + 4]);
  __builtin_amdgcn_wave_barrier();
}

__device__ inline float red_finish(const float4& r0, const float4& r1) {
  return group8_sum(((r0.x + r0.y) + (r0.z + r0.w)) + ((r1.x + r1.y) + (r1.z + r1.w)));
}

__device__ inline float row_reduce9(const float (&g)[9], bool b3, bool b2, bool b1, bool b0) {
  float a[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) a[j] = bfly<0x140>(g[j], g[4 + j], b3);  // row_mirror
  float s8 = g[8] + dpp_read<0x140>(g[8]);
  float c[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) c[j] = bfly<0x141>(a[j], a[2 + j], b2);  // row_half_mirror
  s8 += dpp_read<0x141>(s8);
  const float d = bfly<0x1B>(c[0], c[1], b1);                             // quad_perm [3,2,1,0]
  s8 += dpp_read<0x1B>(s8);
  return bfly<0xB1>(d, s8, b0);                                           // quad_perm [1,0,3,2]
}


// Minimum over the rectangle [x0, x1] x [y0, y1] of f(x, y) = a x^2 + 2 b x y + c y^2 (positive
// definite), with nba = -b/a and nbc = -b/c precomputed.  Float; callers add a margin that covers
// its rounding.
__device__ inline float rect_min_quadratic(float a, float b, float c, float nba, float nbc, float x0, float x1,
                                           float y0, float y1) {
  if (x0 <= 0.0f && 0.0f <= x1 && y0 <= 0.0f && 0.0f <= y1) return 0.0f;
  float m = 3.0e38f;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float x = e ? x1 : x0;  // vertical edge: best y = -b x / c, clamped (median of three)
    const float y = __builtin_amdgcn_fmed3f(nbc * x, y0, y1);
    m = fminf(m, fmaf(a * x, x, y * fmaf(2.0f * b, x, c * y)));
    const float yy = e ? y1 : y0;  // horizontal edge
    const float xx = __builtin_amdgcn_fmed3f(nba * yy, x0, x1);
    m = fminf(m, fmaf(a * xx, xx, yy * fmaf(2.0f * b, xx, c * yy)));
  }
  return m;
}

// Quadrants (8x8 pixel blocks) of a tile that can hold a pixel where the Gaussian reaches
// alpha >= 1/255.  First the padded rectangle u +- eu, v +- ev; then, for quadrants that pass,
// the minimum of the exponent's quadratic form over the quadrant's pixel-centre rectangle.  The
// margin exceeds, tenfold or more, both the compositor's float evaluation error of the exponent
// (rounding of products and of du, dv) and the rounding of this test, so no contributing pixel
// is ever skipped.  Quadrants whose horizontal span reaches the +-W/2 wrap point keep the
// rectangle test only.
// Only the quadrants in `sel` (uniform) are tested; the others read as not reached.
template <int TILE>
__device__ inline uint32_t quadrant_mask(const Rec& r, int tx0, int ty0, float Wf, float half, uint32_t sel = ~0u) {
  constexpr int QPR = TILE / 8;
  const float u = r.r0.x, v = r.r0.y, eu = r.r1.w, ev = r.r2.w;
  // inverse covariance [[a, b], [b, c]] = 2 L^T L of the stored factor
  const float l0 = r.r0.z, l1 = r.r0.w, l2 = r.r1.x;
  const float a = 2.0f * l0 * l0, b = 2.0f * l0 * l1, c = 2.0f * fmaf(l1, l1, l2 * l2);
  const float nba = -b * __builtin_amdgcn_rcpf(a), nbc = -b * __builtin_amdgcn_rcpf(c);
  const float aa = fabsf(a), ab = fabsf(b), ac = fabsf(c);
  const float k2 = -2.0f * r.r1.z;
  const bool all_cols = eu + 3.5f >= half;
  uint32_t mask = 0;
#pragma unroll
  for (int q = 0; q < QPR * QPR; ++q) {
    if (!((sel >> q) & 1u)) continue;
    const float qcx = (float)(tx0 + (q % QPR) * 8 + 4);
    const float qcy = (float)(ty0 + (q / QPR) * 8 + 4);
    float du = qcx - u;
    if (du >= half) du -= Wf;
    else if (du < -half) du += Wf;
    const float dy = qcy - v;
    bool hit = fabsf(dy) <= ev + 3.5f && (all_cols || fabsf(du) <= eu + 3.5f);
    if (hit && fabsf(du) + 4.0f < half) {
      const float X = fabsf(du) + 3.5f, Y = fabsf(dy) + 3.5f;
      const float tmax = fmaf(aa * X, X, Y * fmaf(2.0f * ab, X, ac * Y));
      const float gmax = 2.0f * fmaf(aa + ab, X, (ab + ac) * Y);
      const float margin = fmaf(1e-5f, tmax, fmaf(1e-2f, gmax, fmaf(1e-4f, k2, 1e-6f)));
      hit = rect_min_quadratic(a, b, c, nba, nbc, du - 3.5f, du + 3.5f, dy - 3.5f, dy + 3.5f) <= k2 + margin;
    }
    mask |= hit ? (1u << q) : 0u;
  }
  return mask;
}

// Horizontal offset wrapped into [-W/2, W/2) without branches.
__device__ inline float wrap_du(float du, float Wf, float half) {
  du = du >= half ? du - Wf : du;
  return du < -half ? du + Wf : du;
}

// Stage `cnt` records of a tile list into LDS (entry e <- list position first + dir * e) and
// build, for every wavefront (one per 8x8 quadrant, one pixel per lane), the order-preserving
// list of entries whose footprint reaches its pixels.  Counts per list are returned in nq[]
// (identical in every thread).
template <int TILE, int BATCH>
struct Stage {
  static constexpr int N = TILE * TILE;  // threads
  static constexpr int NQ = (TILE / 8) * (TILE / 8);  // lists = wavefronts
  static constexpr int NW = N / kWave;
  static_assert(NQ == NW, "one list per wavefront");
  float4 s0[BATCH];
  float4 s1[BATCH];
  float4 s2[BATCH];
  uint32_t sid[BATCH];
  float dep[BATCH];  // sort depths (staged only for the expected-depth output)
  uint8_t list[NQ][BATCH];
  uint32_t wcnt[NW][NQ];  // per-wavefront counts, then (in place) exclusive prefix over wavefronts
  uint32_t tot[NQ];
};

// The culling masks travel from the forward to the backward: the forward stores, per list position,
// the quadrants of the reverse compositor's task in which some of its pixels reached the entry (see
// s_used; narrower than the footprint's) into the pair buffer the sort leaves unused, and the
// backward loads them instead of evaluating the footprint again: one byte per position, in byte
// planes at 16x16 blocks (the task's plane, see task_block).  The mask is written after the forward
// walks each batch.  The backward reads only list positions before its tile's last contributor,
// all of which the forward staged.
enum QuadMaskMode { kMaskEval = 0, kMaskLoad = 2 };

// Returns whether the seam wrap is the identity for every staged entry (uniform).
template <int TILE, int BATCH, int QM = kMaskEval>
__device__ inline bool stage_batch(Stage<TILE, BATCH>& S, const uint32_t* __restrict__ pair_items,
                                   const Rec* __restrict__ rec, uint32_t first, int dir, int cnt, int tx0, int ty0,
                                   float Wf, float half, int (&nq)[Stage<TILE, BATCH>::NQ],
                                   const float* __restrict__ depth = nullptr,
                                   const uint8_t* __restrict__ qmask_in = nullptr) {
  using St = Stage<TILE, BATCH>;
  const int t = threadIdx.x, ln = t & (kWave - 1), wv = t >> 6;
  const uint64_t below = ln == 0 ? 0ull : (~0ull >> (kWave - ln));
#pragma unroll
  for (int q = 0; q < St::NQ; ++q) nq[q] = 0;
  bool nowrap = true, all_nowrap = true;
  for (int r0 = 0; r0 < cnt; r0 += St::N) {
    const int e = r0 + t;
    uint32_t m = 0;
    if (e < cnt) {
      const uint32_t pos = first + dir * e;
      const uint32_t item = pair_items[pos];
      const Rec r = rec[item];
      S.s0[e] = r.r0;
      // the fourth word (the half extent, needed only for the mask below) carries whether every
      // pixel centre of the tile lies within W/2 - 1 of u: the seam wrap is then the identity
      const float reach = fabsf((float)tx0 + 0.5f * (float)TILE - r.r0.x) + 0.5f * (float)TILE + 1.0f;
      nowrap = nowrap && reach < half;
      // staged as (l2, p_min, opacity, no-wrap flag): the accept test reads its two words with one
      // 8-byte LDS load at an immediate offset
      S.s1[e] = make_float4(r.r1.x, r.r1.z, r.r1.y, reach < half ? 1.0f : 0.0f);
      S.s2[e] = r.r2;
      S.sid[e] = item;
      if (depth) S.dep[e] = depth[item];
      if constexpr (QM == kMaskLoad) {
        m = qmask_in[pos];
      } else {
        m = quadrant_mask<TILE>(r, tx0, ty0, Wf, half);
      }
    }
    uint32_t within[St::NQ];
#pragma unroll
    for (int q = 0; q < St::NQ; ++q) {
      const uint64_t bq = __builtin_amdgcn_ballot_w64((m >> q) & 1u);
      within[q] = __popcll(bq & below);
      if (ln == 0) S.wcnt[wv][q] = __popcll(bq);
    }
    __syncthreads();
    if constexpr (St::NW > 1) {
      // thread q turns list q's per-wavefront counts into exclusive prefixes
      if (t < St::NQ) {
        uint32_t run = 0;
#pragma unroll
        for (int w = 0; w < St::NW; ++w) {
          const uint32_t c = S.wcnt[w][t];
          S.wcnt[w][t] = run;
          run += c;
        }
        S.tot[t] = run;
      }
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < St::NQ; ++q) {
      const int pre = St::NW > 1 ? (int)S.wcnt[wv][q] : 0;
      const int tot = St::NW > 1 ? (int)S.tot[q] : (int)S.wcnt[0][q];
      if ((m >> q) & 1u) S.list[q][nq[q] + pre + (int)within[q]] = (uint8_t)e;
      nq[q] += tot;
    }
    all_nowrap = __syncthreads_and(nowrap) != 0;
  }
  return all_nowrap;
}

// COUNT: also record the per-pixel work counters read by odgs_debug_pixel_counts (a separate
// instantiation, so the production forward carries no counting instructions).
// DEPTH: also write the alpha-weighted sort depth sum_j alpha_j T_j d_j of every pixel.
template <int TILE, int BATCH, bool COUNT, bool DEPTH>
__global__ __launch_bounds__(TILE* TILE) void render_fwd_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items, const Rec* __restrict__ rec,
    float* __restrict__ out_rgb, float* __restrict__ out_T, float* __restrict__ ws_T, int32_t* __restrict__ ws_last,
    int32_t* __restrict__ ws_ncontrib, int32_t* __restrict__ ws_neval, int32_t* __restrict__ ws_lasteval, float bg0,
    float bg1, float bg2, const float* __restrict__ depth, float* __restrict__ out_depth, uint8_t* __restrict__ qmask,
    int64_t qplane, TileSched sc) {
  using St = Stage<TILE, BATCH>;
  constexpr int N = St::N;
  __shared__ St S;
  // s_used[q][e]: some still-compositing pixel of quadrant q reaches entry e of the batch being
  // walked.  For list positions before a pixel's last contributor, that test here and the
  // backward's are the same float decision, so these quadrants include every one whose pixels the
  // backward must visit the entry for (and little else); that mask, in the backward's
  // granularity, is what the backward loads.
  __shared__ uint8_t s_used[St::NQ][BATCH];
  mark_forward(sc);
  __shared__ uint32_t s_claim;
  uint32_t round = 0;
  for (int g; (g = claim_tile(sc, round, &s_claim)) >= 0;) {
    const int v = view_of_tile(vt, g);
    const int W = vt.W[v], H = vt.H[v];
    const int ntx = W / TILE;
    const int lt = g - vt.tile_base[v];
    const int tx0 = (lt % ntx) * TILE, ty0 = (lt / ntx) * TILE;
    int lx, ly;
    local_pixel<TILE>(threadIdx.x, lx, ly);
    const int x = tx0 + lx, y = ty0 + ly;
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // this wavefront's quadrant (uniform)
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float Wf = (float)W, half = wrap_half(vt, v);  // no seam in pinhole views
    const uint2 rg = ranges[g];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f;
    int last = 0, ncontrib = 0, nev = 0, lastev = 0;
    // 0 while the pixel composites, NaN once it has stopped: added to the exponent's sum of squares
    // it makes the accept compare itself false for every later Gaussian (with 0 the sum is the same
    // float), so the wavefront's ballots are of single compares
    float qstop = 0.0f;
    // writes the masks of the batch walked last (after a barrier) and clears s_used for the next
    auto flush_used = [&](uint32_t first, int n_walked) {
      for (int e = threadIdx.x; e < BATCH; e += N) {
        if (e < n_walked) {
          uint32_t mq = 0;
#pragma unroll
          for (int q = 0; q < St::NQ; ++q) mq |= s_used[q][e] ? (1u << q) : 0u;
          if constexpr (TILE >= 32) {
            // the reverse compositor takes each 16x16 block b = 2 by + bx of a 32x32 tile as a
            // task: its four quadrants' bits go to byte plane b
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int q0 = 8 * (b >> 1) + 2 * (b & 1);  // quadrant (2 bx, 2 by) of the 4x4 grid
              qmask[(int64_t)b * qplane + first + e] =
                  (uint8_t)(((mq >> q0) & 3u) | (((mq >> (q0 + 4)) & 3u) << 2));
            }
          } else {
            qmask[first + e] = (uint8_t)mq;
          }
        }
#pragma unroll
        for (int q = 0; q < St::NQ; ++q) s_used[q][e] = 0;
      }
    };
    uint32_t walked_base = 0;
    int walked_cnt = 0;
    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
      const bool all_done = __syncthreads_count(!(qstop == 0.0f)) == N;
      flush_used(walked_base, walked_cnt);
      walked_cnt = 0;
      if (all_done) break;
      const int cnt = (int)min((uint32_t)BATCH, rg.y - base);
      int nq[St::NQ];
      const bool nowrap =
          stage_batch<TILE, BATCH>(S, pair_items, rec, base, 1, cnt, tx0, ty0, Wf, half, nq, DEPTH ? depth : nullptr);
      const int n = __builtin_amdgcn_readfirstlane(nq[wq]);
      // one list walk, instantiated without the seam wrap for batches where it is the identity
      auto walk = [&](auto wrapc) {
      for (int i = 0; i < n; ++i) {
        if (__builtin_amdgcn_ballot_w64(qstop == 0.0f) == 0ull) break;  // uniform: every pixel has finished
        const int k = S.list[wq][i];
        const float4 a = S.s0[k];
        const float4 b = S.s1[k];
        const float du = decltype(wrapc)::value ? wrap_du(px - a.x, Wf, half) : px - a.x;
        const float dv = py - a.y;
        const float t1 = fmaf(a.z, du, a.w * dv), t2 = b.x * dv;
        const float power = -fmaf(t1, t1, fmaf(t2, t2, qstop));
        if (COUNT) nev += qstop == 0.0f ? 1 : 0;
        // alpha >= 1/255 (power <= 0 always: a sum of squares; NaN once stopped)
        const bool ok = power >= b.y;
        if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
        // some pixel of this quadrant reaches the entry (it is accepted there unless that pixel
        // stops at it, in which case the backward does not need it for that pixel: a superset)
        s_used[wq][k] = 1;
        const float alpha = fminf(b.z * __expf(power), kAlphaMax);
        const float Tn = T * (1.0f - alpha);
        const bool acc = ok && !(Tn < kTStop);
        qstop = ok != acc ? __builtin_nanf("") : qstop;  // stop: reached, but T would drop below 1e-4
        const float4 c = S.s2[k];
        const float w = (acc ? alpha : 0.0f) * T;  // (a select of the product compiles to a branch here)
        C0 = fmaf(w, c.x, C0);
        C1 = fmaf(w, c.y, C1);
        C2 = fmaf(w, c.z, C2);
        if (DEPTH) D = D + w * S.dep[k];
        T = acc ? Tn : T;
        last = acc ? (int)(base - rg.x) + k + 1 : last;
        if (COUNT) {
          lastev = acc ? nev : lastev;
          ncontrib += acc ? 1 : 0;
        }

      }
      };
      if (nowrap)
        walk(std::false_type{});
      else
        walk(std::true_type{});
      walked_base = base;
      walked_cnt = cnt;
    }
    __syncthreads();
    flush_used(walked_base, walked_cnt);
    const int64_t plane = (int64_t)W * H;
    const int64_t pix = (int64_t)y * W + x;
    float* img = out_rgb + 3 * vt.pix_base[v];
    img[pix] = fmaf(T, bg0, C0);
    img[plane + pix] = fmaf(T, bg1, C1);
    img[2 * plane + pix] = fmaf(T, bg2, C2);
    const int64_t gp = vt.pix_base[v] + pix;
    ws_T[gp] = T;
    ws_last[gp] = last;
    if (COUNT) {
      ws_ncontrib[gp] = ncontrib;
      ws_neval[gp] = nev;
      ws_lasteval[gp] = lastev;
    }
    if (DEPTH) out_depth[gp] = D;
    if (out_T) out_T[gp] = T;
  }
}

// Forward compositing of a 16x16 tile by one wavefront, four pixels per lane (lane l holds pixel
// (l % 8, l / 8) of each quadrant): the tile's list is staged once with each entry's quadrant mask
// (the footprint test of the one-pixel forward), and an entry is evaluated only for the quadrants
// it can reach and whose pixels still composite.  The quadrants in which some pixel reached an
// entry are handed to the backward as in the one-pixel forward.  A quadrant task of a split tile
// (see TileSched) runs the same code with its one quadrant selected, and hands its masks over in
// the byte plane of its quadrant (plane q at byte offset q * qplane; whole tiles use plane 0).
// The 16x16 pixel block a task composites: its origin (bx0, by0), its quadrants (`sel`, updated)
// and the byte plane of its culling masks.  BIN = 16: the tile, or one quadrant of a split tile
// (plane q); BIN = 32: part p of the tile, the 16x16 block p = 2 by + bx with all four quadrants
// (plane p).
template <int BIN>
__device__ inline void task_block(const ViewTable& vt, int v, int g, uint32_t& sel, int& bx0, int& by0, int& plane) {
  const int ntx = vt.W[v] / BIN;
  const int lt = g - vt.tile_base[v];
  bx0 = (lt % ntx) * BIN;
  by0 = (lt / ntx) * BIN;
  plane = sel == 0xFu ? 0 : __builtin_ctz(sel);
  if constexpr (BIN == 32) {
    bx0 += 16 * (plane & 1);
    by0 += 16 * (plane >> 1);
    sel = 0xFu;
  } else {
    static_assert(BIN == 16, "blocks of 16x16 pixels in tiles of 16 or 32");
  }
}

template <int BATCH>
struct FwdStage4 {
  float4 s0[BATCH];
  float4 s1[BATCH];
  float4 s2[BATCH];
  uint16_t list[BATCH];  // entry index | quadrant mask << 8
  uint8_t used[BATCH];
};

template <int BIN, int BATCH>
__global__ __launch_bounds__(kWave) void render_fwd4_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items, const Rec* __restrict__ rec,
    float* __restrict__ out_rgb, float* __restrict__ out_T, float* __restrict__ ws_T, int32_t* __restrict__ ws_last,
    float bg0, float bg1, float bg2, uint8_t* __restrict__ qmask, int64_t qplane, TileSched sc) {
  constexpr int TILE = 16;
  __shared__ FwdStage4<BATCH> S;
  const int nsplit = forward_split(sc);
  mark_forward(sc, nsplit);
  __shared__ uint32_t s_claim;
  uint32_t round = 0, sel = 0;
  const int lane = threadIdx.x;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  for (int g; (g = claim_task(sc, nsplit, round, &s_claim, sel)) >= 0;) {
    const int v = view_of_tile(vt, g);
    const int W = vt.W[v], H = vt.H[v];
    int tx0, ty0, pl;
    task_block<BIN>(vt, v, g, sel, tx0, ty0, pl);
    const int x = tx0 + (lane & 7), y = ty0 + (lane >> 3);
    const float px0 = (float)x + 0.5f, px1 = (float)(x + 8) + 0.5f;
    const float py0 = (float)y + 0.5f, py1 = (float)(y + 8) + 0.5f;
    const float Wf = (float)W, half = wrap_half(vt, v);
    const uint2 rg = ranges[g];
    float T[4], C0[4], C1[4], C2[4], qstop[4];  // qstop: 0 while compositing, NaN once stopped
    int last[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T[q] = 1.0f;
      C0[q] = C1[q] = C2[q] = 0.0f;
      qstop[q] = 0.0f;
      last[q] = 0;
    }
    uint32_t alive = sel;  // selected quadrants with a pixel still compositing (uniform)
    uint8_t* qm = qmask + (int64_t)pl * qplane;
    for (uint32_t base = rg.x; base < rg.y && alive != 0u; base += BATCH) {
      const int cnt = (int)min((uint32_t)BATCH, rg.y - base);
      int n = 0;
      for (int r0 = 0; r0 < cnt; r0 += kWave) {
        const int e = r0 + lane;
        uint32_t m = 0;
        if (e < cnt) {
          const Rec r = rec[pair_items[base + e]];
          S.s0[e] = r.r0;
          const float reach = fabsf((float)tx0 + 0.5f * (float)TILE - r.r0.x) + 0.5f * (float)TILE + 1.0f;
          S.s1[e] = make_float4(r.r1.x, r.r1.z, r.r1.y, reach < half ? 1.0f : 0.0f);
          S.s2[e] = r.r2;
          S.used[e] = 0;
          m = quadrant_mask<TILE>(r, tx0, ty0, Wf, half, sel);
        }
        const uint64_t bl = __builtin_amdgcn_ballot_w64(m != 0u);
        if (m != 0u) S.list[n + __popcll(bl & below)] = (uint16_t)(e | (m << 8));
        n += __popcll(bl);
      }
      __syncthreads();
      uint32_t kmn = S.list[0];  // the next entry's list word, read one entry ahead
      for (int i = 0; i < n; ++i) {
        const uint32_t km = __builtin_amdgcn_readfirstlane(kmn);
        kmn = S.list[min(i + 1, n - 1)];
        const int k = (int)(km & 0xFFu);
        const uint32_t mq = (km >> 8) & alive;
        if (mq == 0u) continue;  // uniform
        const float4 a = S.s0[k];
        const float4 b = S.s1[k];
        const bool wrap = __builtin_amdgcn_readfirstlane(__float_as_int(b.w)) == 0;  // uniform
        float du0 = px0 - a.x, du1 = px1 - a.x;
        if (wrap) {
          du0 = wrap_du(du0, Wf, half);
          du1 = wrap_du(du1, Wf, half);
        }
        uint32_t used = 0;
        const float4 c = S.s2[k];  // once per entry, not per accepting quadrant: forward 0.81 -> 0.78 ms
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!((mq >> q) & 1u)) continue;  // uniform
          const float dv = (q >> 1 ? py1 : py0) - a.y;
          const float du = q & 1 ? du1 : du0;
          const float t1 = fmaf(a.z, du, a.w * dv), t2 = b.x * dv;
          const float power = -fmaf(t1, t1, fmaf(t2, t2, qstop[q]));
          const bool ok = power >= b.y;  // alpha >= 1/255 (NaN once the pixel has stopped)
          const uint64_t bok = __builtin_amdgcn_ballot_w64(ok);
          if (bok == 0ull) continue;  // uniform
          used |= 1u << q;
          const float alpha = fminf(b.z * __expf(power), kAlphaMax);
          const float Tn = T[q] * (1.0f - alpha);
          const bool acc = ok && !(Tn < kTStop);
          qstop[q] = ok != acc ? __builtin_nanf("") : qstop[q];  // stop: reached, but T would drop below 1e-4
          const float w = (acc ? alpha : 0.0f) * T[q];
          C0[q] = fmaf(w, c.x, C0[q]);
          C1[q] = fmaf(w, c.y, C1[q]);
          C2[q] = fmaf(w, c.z, C2[q]);
          T[q] = acc ? Tn : T[q];
          last[q] = acc ? (int)(base - rg.x) + k + 1 : last[q];
        }
        if (lane == 0 && used) S.used[k] = (uint8_t)used;
      }
      // quadrants whose pixels have all stopped (taken once per batch: within a batch a stopped
      // quadrant costs its test per entry, which no longer reaches any pixel)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (((alive >> q) & 1u) && __builtin_amdgcn_ballot_w64(qstop[q] == 0.0f) == 0ull) alive &= ~(1u << q);
      __syncthreads();
      // the backward's masks for this batch: the quadrants in which some pixel reached each entry
      for (int e = lane; e < cnt; e += kWave) qm[base + e] = S.used[e];
      __syncthreads();
    }
    // entries past the point where every pixel stopped were never reached: their masks stay as
    // the binning left them, and the backward (which stops at each tile's last contributor) never
    // reads them
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((sel >> q) & 1u)) continue;
      const int64_t pix = (int64_t)(y + 8 * (q >> 1)) * W + x + 8 * (q & 1);
      float* img = out_rgb + 3 * vt.pix_base[v];
      const int64_t plane = (int64_t)W * H;
      img[pix] = fmaf(T[q], bg0, C0[q]);
      img[plane + pix] = fmaf(T[q], bg1, C1[q]);
      img[2 * plane + pix] = fmaf(T[q], bg2, C2[q]);
      const int64_t gp = vt.pix_base[v] + pix;
      ws_T[gp] = T[q];
      ws_last[gp] = last[q];
      if (out_T) out_T[gp] = T[q];
    }
  }
}

// Reverse compositing state of one pixel (back to front from its last contributor).
struct BwdPixel {
  float T, DS, dl0, dl1, dl2;  // DS = dL/dC . (colour of everything behind, incl. background)
  int last;
};

// The position and shape sums are taken in the footprint's whitened coordinates t = L d
// (t1 = l0 du + l1 dv, t2 = l2 dv, L = [[l0, l1], [0, l2]] the record's factor of Sigma^-1 / 2, so
// power = -|t|^2): per pixel dpow * t and dpow * t t^T, whose entries are all of the same order for
// any footprint shape.  With h = L^T t = Sigma^-1 d / 2, d power / d(u, v) = 2 h and
// d power / d Sigma_2D = 2 h h^T, so the per-tile sums S_t = sum dpow t and Z = sum dpow t t^T map
// exactly to g_(u,v) = 2 L^T S_t and g_Sigma = 2 L^T Z L.  That map is applied once per (Gaussian,
// tile) in double at the flush.  (Summing dpow h h^T directly in float loses the long axis of a
// needle-like footprint: there h lies almost along the short axis and the long-axis component of
// h h^T sits ~1e5 below the rounding of the short one.)
template <int NS, int B>
__device__ inline double acc_total(const float (&acc)[NS][9][B], int q, int t) {
  double s = (double)acc[0][q][t];
#pragma unroll
  for (int w = 1; w < NS; ++w) s += (double)acc[w][q][t];
  return s;
}

// Value q of an entry's 2D-gradient record (layout of g2d) from its per-wavefront sums; a, b: the
// entry's staged record words (l0 = a.z, l1 = a.w, l2 = b.x).
template <int NS, int B>
__device__ inline double g2d_flush_value(const float (&acc)[NS][9][B], int q, int t, const float4& a, const float4& b) {
  const double l0 = a.z, l1 = a.w, l2 = b.x;
  switch (q) {
    case 0: return 2.0 * l0 * acc_total(acc, 0, t);
    case 1: return 2.0 * (l1 * acc_total(acc, 0, t) + l2 * acc_total(acc, 1, t));
    case 2: return 2.0 * (l0 * l0) * acc_total(acc, 2, t);
    case 3: return 4.0 * l0 * (l1 * acc_total(acc, 2, t) + l2 * acc_total(acc, 3, t));
    case 4: {
      const double z11 = acc_total(acc, 2, t), z12 = acc_total(acc, 3, t), z22 = acc_total(acc, 4, t);
      return 2.0 * ((l1 * l1) * z11 + 2.0 * (l1 * l2) * z12 + (l2 * l2) * z22);
    }
    default: return acc_total(acc, q, t);
  }
}

// One pixel's contribution of a Gaussian to the nine per-tile sums (added to gq when ADD, else
// written; slots 0..4 in whitened coordinates as above), and the pixel's recursion step.  `ok`:
// the Gaussian contributed to this pixel; t1 = l0 du + l1 dv, t2 = l2 dv.
template <bool ADD>
__device__ inline void bwd_pixel_step(BwdPixel& P, bool ok, float power, float t1, float t2, const float4& a,
                                      const float4& b, const float4& c, float (&gq)[9]) {
  const float G = __expf(power);
  const float araw = b.z * G;
  const bool live = ok && !(araw > kAlphaMax);  // contributes and unclamped: alpha depends on the inputs
  // alpha = 0 where the Gaussian does not contribute, so its weight below is 0 without a select
  const float alpha = ok ? fminf(araw, kAlphaMax) : 0.0f;
  const float inv_om = __builtin_amdgcn_rcpf(1.0f - alpha);
  // transmittance in front of this Gaussian; where it does not contribute alpha = 0 and the
  // reciprocal of 1 is exactly 1 (powers of two are exact), so T is unchanged without a select
  P.T = P.T * inv_om;
  const float wk = alpha * P.T;
  const float dc = fmaf(P.dl0, c.x, fmaf(P.dl1, c.y, P.dl2 * c.z));  // dL/dC . colour
  const float dL_da = fmaf(dc, P.T, -P.DS * inv_om);
  P.DS = fmaf(dc, wk, P.DS);
  const float dla = live ? dL_da : 0.0f;
  const float dpow = dla * alpha;
  const float g0 = dpow * t1, g1 = dpow * t2;
  // values 2..8 are products x_q y_q (fused into the running sums when adding)
  const float x[7] = {g0, g0, g1, dla, wk, wk, wk}, y[7] = {t1, t2, t2, G, P.dl0, P.dl1, P.dl2};
  gq[0] = ADD ? gq[0] + g0 : g0;
  gq[1] = ADD ? gq[1] + g1 : g1;
#pragma unroll
  for (int q = 0; q < 7; ++q) gq[2 + q] = ADD ? fmaf(x[q], y[q], gq[2 + q]) : x[q] * y[q];
}

// g2d layout: [items][9] = d/du, d/dv, d/dS_uu, d/dS_uv, d/dS_vv, d/dopacity, d/dr, d/dg,
// d/db(colour), where Sigma_2D = [[S_uu, S_uv], [S_uv, S_vv]] (S_uv the shared off-diagonal),
// formed per (Gaussian, tile) from the whitened-coordinate sums (g2d_flush_value).
template <int TILE, int BATCH>
__global__ __launch_bounds__(TILE* TILE) void render_bwd_kernel(ViewTable vt, const uint2* __restrict__ ranges,
                                                                const uint32_t* __restrict__ pair_items,
                                                                const Rec* __restrict__ rec, const float* __restrict__ ws_T,
                                                                const int32_t* __restrict__ ws_last,
                                                                const float* __restrict__ dL_drgb, double* __restrict__ g2d,
                                                                int64_t items, float bg0, float bg1, float bg2,
                                                                const uint8_t* __restrict__ qmask, TileSched sc) {
  static_assert(TILE == 8, "tiles of 16 and 32 take the four-pixel kernel");
  using St = Stage<TILE, BATCH>;
  constexpr int N = St::N;
  // One wavefront per 8x8 tile, owning a slot per (value, entry) (the slot-set logic is written
  // for up to four wavefronts, whose sets are summed at the flush, so no LDS atomics).
  constexpr bool kSlots = St::NW <= 4;
  constexpr int NS = kSlots ? St::NW : 1;
  __shared__ St S;
  __shared__ float acc[NS][9][BATCH + 1];  // padded rows: the nine slot writes hit nine banks
  __shared__ float red[kSlots ? St::NW : 1][8][kRedStride];  // per-wavefront reduction scratch
  __shared__ int smax;
  if (forward_is_stale(sc)) return;  // uniform
  __shared__ uint32_t s_claim;
  uint32_t round = 0;
  for (int g; (g = claim_tile(sc, round, &s_claim)) >= 0;) {
    const int v = view_of_tile(vt, g);
    const int W = vt.W[v], H = vt.H[v];
    const int ntx = W / TILE;
    const int lt = g - vt.tile_base[v];
    const int tx0 = (lt % ntx) * TILE, ty0 = (lt / ntx) * TILE;
    int lx, ly;
    local_pixel<TILE>(threadIdx.x, lx, ly);
    const int x = tx0 + lx, y = ty0 + ly;
    const int lane = threadIdx.x & (kWave - 1);
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int slot = (int)((kRowSlot >> (4 * (lane & 15))) & 0xF);
    const float px = (float)x + 0.5f, py = (float)y + 0.5f;
    const float Wf = (float)W, half = wrap_half(vt, v);  // no seam in pinhole views
    const uint2 rg = ranges[g];
    const int64_t plane = (int64_t)W * H;
    const int64_t pix = (int64_t)y * W + x;
    const int64_t gp = vt.pix_base[v] + pix;
    const float* dimg = dL_drgb + 3 * vt.pix_base[v];
    BwdPixel P;
    P.dl0 = dimg[pix], P.dl1 = dimg[plane + pix], P.dl2 = dimg[2 * plane + pix];
    P.T = ws_T[gp];
    P.last = ws_last[gp];
    // dL/dC . (colour of everything behind, incl. background): the only way the colour behind a
    // Gaussian enters its alpha gradient, so one scalar replaces the three channels
    P.DS = P.T * fmaf(P.dl0, bg0, fmaf(P.dl1, bg1, P.dl2 * bg2));
    // largest `last` of the wavefront (uniform) and of the workgroup
    int wmax = P.last;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off));
    wmax = __builtin_amdgcn_readfirstlane(wmax);
    if (threadIdx.x == 0) smax = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&smax, wmax);
    __syncthreads();
    const int end_all = smax;
    for (int end = end_all; end > 0; end -= BATCH) {
      const int cnt = min(BATCH, end);
      for (int t = threadIdx.x; t < cnt; t += N) {
#pragma unroll
        for (int w = 0; w < NS; ++w)
#pragma unroll
          for (int q = 0; q < 9; ++q) acc[w][q][t] = 0.0f;
      }
      int nq[St::NQ];
      // entry e is list position end - 1 - e (back to front)
      stage_batch<TILE, BATCH, kMaskLoad>(S, pair_items, rec, rg.x + end - 1, -1, cnt, tx0, ty0, Wf, half, nq, nullptr,
                                             qmask);
      const int n = __builtin_amdgcn_readfirstlane(nq[wq]);
      bool pend = false;  // an accepted entry whose values 0..7 still wait in red (uniform)
      int pk = 0;
      // software pipeline: the next entry's list index and records are read while this one is
      // processed, taking two LDS round trips off each iteration's dependency chain
      int kn = n > 0 ? S.list[wq][0] : 0;  // entries 0..n-1 of the list are valid
      float4 an = S.s0[kn], bn = S.s1[kn];
      for (int i = 0; i < n; ++i) {
        const int k = __builtin_amdgcn_readfirstlane(kn);  // uniform entry index
        const float4 a = an, b = bn;
        kn = S.list[wq][min(i + 1, n - 1)];
        an = S.s0[kn];
        bn = S.s1[kn];
        const int jrel = end - 1 - k;
        if (jrel >= wmax) continue;  // uniform: behind every contributor of this wavefront
        const float du = wrap_du(px - a.x, Wf, half);
        const float dv = py - a.y;
        const float t1 = fmaf(a.z, du, a.w * dv), t2 = b.x * dv;
        const float power = -fmaf(t1, t1, t2 * t2);
        const bool ok = jrel < P.last && !(power > 0.0f || power < b.y);
        if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
        float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
        if (kSlots && pend) red_read(red[wq], lane, r0, r1);  // previous accepted entry's values
        const float4 c = S.s2[k];
        float gq[9];
        bwd_pixel_step<false>(P, ok, power, t1, t2, a, b, c, gq);
        if constexpr (kSlots) {
          if (pend) {
            const float sj = red_finish(r0, r1);
            if ((lane & 7) == 0) acc[wq][lane >> 3][pk] = sj;
          }
          red_write(red[wq], gq, lane);
          const float s8 = wave_sum(gq[8]);
          if (lane == 1) acc[wq][8][k] = s8;
          pend = true;
          pk = k;
        } else {
          const float rs = row_reduce9(gq, lane & 8, lane & 4, lane & 2, lane & 1);
          if (slot < 9) atomicAdd(&acc[0][slot][k], rs);  // 9 lanes per row, 4 rows: one LDS atomic
        }
      }
      if (kSlots && pend) {
        float4 r0, r1;
        red_read(red[wq], lane, r0, r1);
        const float sj = red_finish(r0, r1);
        if ((lane & 7) == 0) acc[wq][lane >> 3][pk] = sj;
      }
      __syncthreads();
      // nine consecutive lanes carry one entry's nine values, so one atomic instruction covers
      // about seven items' contiguous 72-byte gradient records instead of 64 scattered lines
      for (int x = threadIdx.x; x < 9 * cnt; x += N) {
        const int t = x / 9, q = x - 9 * t;
        const double s = g2d_flush_value(acc, q, t, S.s0[t], S.s1[t]);
        if (s != 0.0) unsafeAtomicAdd(&g2d[(int64_t)S.sid[t] * 9 + q], s);
      }
      __syncthreads();
    }
  }
}

// Reverse compositing of a 16x16 tile by one wavefront, four pixels per lane (lane l holds pixel
// (l % 8, l / 8) of each quadrant): the four quadrants' contributions to an entry are added in
// registers and reduced across lanes once, and a quadrant the forward's pixels did not reach
// (its bit in the staged mask) costs nothing for that entry.
template <int BATCH>
struct Stage4 {
  float4 s0[BATCH];
  float4 s1[BATCH];
  float4 s2[BATCH];
  uint32_t sid[BATCH];
  uint16_t list[BATCH];  // entry index | quadrant mask << 8
};

template <int BIN, int BATCH>
__global__ __launch_bounds__(kWave) void render_bwd4_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items, const Rec* __restrict__ rec,
    const float* __restrict__ ws_T, const int32_t* __restrict__ ws_last, const float* __restrict__ dL_drgb,
    double* __restrict__ g2d, int64_t items, float bg0, float bg1, float bg2, const uint8_t* __restrict__ qmask,
    int64_t qplane, TileSched sc) {
  constexpr int TILE = 16;
  __shared__ Stage4<BATCH> S;
  __shared__ float acc[1][9][BATCH + 1];
  if (forward_is_stale(sc)) return;  // uniform
  const int nsplit = reverse_split(sc);
  __shared__ uint32_t s_claim;
  uint32_t round = 0, sel = 0;
  const int lane = threadIdx.x;
  const int slot = (int)((kRowSlot >> (4 * (lane & 15))) & 0xF);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  for (int g; (g = claim_task(sc, nsplit, round, &s_claim, sel)) >= 0;) {
    const int v = view_of_tile(vt, g);
    const int W = vt.W[v], H = vt.H[v];
    int tx0, ty0, pl;
    task_block<BIN>(vt, v, g, sel, tx0, ty0, pl);
    const int x = tx0 + (lane & 7), y = ty0 + (lane >> 3);
    const float px0 = (float)x + 0.5f, px1 = (float)(x + 8) + 0.5f;
    const float py0 = (float)y + 0.5f, py1 = (float)(y + 8) + 0.5f;
    const float Wf = (float)W, half = wrap_half(vt, v);
    const uint2 rg = ranges[g];
    const int64_t plane = (int64_t)W * H;
    const float* dimg = dL_drgb + 3 * vt.pix_base[v];
    BwdPixel P[4];  // quadrant q = 2 * qy + qx
    int wmax = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((sel >> q) & 1u)) {
        P[q].last = 0;  // not this task's: never reached, its other members never read
        continue;
      }
      const int64_t pix = (int64_t)(y + 8 * (q >> 1)) * W + x + 8 * (q & 1);
      const int64_t gp = vt.pix_base[v] + pix;
      P[q].dl0 = dimg[pix], P[q].dl1 = dimg[plane + pix], P[q].dl2 = dimg[2 * plane + pix];
      P[q].T = ws_T[gp];
      P[q].last = ws_last[gp];
      P[q].DS = P[q].T * fmaf(P[q].dl0, bg0, fmaf(P[q].dl1, bg1, P[q].dl2 * bg2));
      wmax = max(wmax, P[q].last);
    }
    const uint8_t* qm = qmask + (int64_t)pl * qplane;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) wmax = max(wmax, __shfl_xor(wmax, off));
    wmax = __builtin_amdgcn_readfirstlane(wmax);
    for (int end = wmax; end > 0; end -= BATCH) {
      const int cnt = min(BATCH, end);
      // stage entries end - 1 - e (back to front) with their quadrant masks; list those reaching
      // any quadrant, in order
      int n = 0;
      for (int r0 = 0; r0 < cnt; r0 += kWave) {
        const int e = r0 + lane;
        uint32_t m = 0;
        if (e < cnt) {
          const uint32_t pos = rg.x + end - 1 - e;
          m = qm[pos] & sel;
          if (m != 0u) {  // records only of the entries the forward's pixels reached
            const uint32_t item = pair_items[pos];
            const Rec r = rec[item];
            S.s0[e] = r.r0;
            const float reach = fabsf((float)tx0 + 0.5f * (float)TILE - r.r0.x) + 0.5f * (float)TILE + 1.0f;
            S.s1[e] = make_float4(r.r1.x, r.r1.z, r.r1.y, reach < half ? 1.0f : 0.0f);
            S.s2[e] = r.r2;
            S.sid[e] = item;
#pragma unroll
            for (int q = 0; q < 9; ++q) acc[0][q][e] = 0.0f;
          }
        }
        const uint64_t bl = __builtin_amdgcn_ballot_w64(m != 0u);
        if (m != 0u) S.list[n + __popcll(bl & below)] = (uint16_t)(e | (m << 8));
        n += __popcll(bl);
      }
      __syncthreads();
      uint32_t kmn = S.list[0];  // the next entry's list word, read one entry ahead
      for (int i = 0; i < n; ++i) {
        const uint32_t km = __builtin_amdgcn_readfirstlane(kmn);
        kmn = S.list[min(i + 1, n - 1)];
        const int k = (int)(km & 0xFFu);
        const int jrel = end - 1 - k;
        const float4 a = S.s0[k];
        const float4 b = S.s1[k];
        const uint32_t mq = km >> 8;
        const bool wrap = __builtin_amdgcn_readfirstlane(__float_as_int(b.w)) == 0;  // uniform
        float du0 = px0 - a.x, du1 = px1 - a.x;
        if (wrap) {
          du0 = wrap_du(du0, Wf, half);
          du1 = wrap_du(du1, Wf, half);
        }
        const float4 c = S.s2[k];
        float gq[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) gq[q] = 0.0f;
        bool any = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!((mq >> q) & 1u)) continue;  // uniform: no pixel of this quadrant reached the entry
          const float dv = (q >> 1 ? py1 : py0) - a.y;
          const float du = q & 1 ? du1 : du0;
          const float t1 = fmaf(a.z, du, a.w * dv), t2 = b.x * dv;
          const float p = -fmaf(t1, t1, t2 * t2);
          const bool ok = jrel < P[q].last && !(p < b.y);
          if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
          bwd_pixel_step<true>(P[q], ok, p, t1, t2, a, b, c, gq);
          any = true;
        }
        if (!any) continue;  // uniform
        const float rs = row_reduce9(gq, lane & 8, lane & 4, lane & 2, lane & 1);
        const float ws = sum_rows(rs);
        if (lane < 16 && slot < 9) acc[0][slot][k] = ws;
      }
      __syncthreads();
      // the listed entries only (the others reached no pixel of this task)
      for (int xq = lane; xq < 9 * n; xq += kWave) {
        const int i = xq / 9, q = xq - 9 * i;
        const int t = S.list[i] & 0xFF;
        const double s = g2d_flush_value(acc, q, t, S.s0[t], S.s1[t]);
        if (s != 0.0) unsafeAtomicAdd(&g2d[(int64_t)S.sid[t] * 9 + q], s);
      }
      __syncthreads();
    }
  }
}

__global__ void debug_records_kernel(const Rec* __restrict__ rec, const float* __restrict__ depth,
                                     const uint32_t* __restrict__ count, int64_t items, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= items) return;
  const Rec r = rec[i];
  float* o = out + i * 12;
  o[0] = r.r0.x; o[1] = r.r0.y; o[2] = r.r0.z; o[3] = r.r0.w;
  o[4] = r.r1.x; o[5] = r.r1.y; o[6] = r.r1.z; o[7] = depth[i];
  o[8] = r.r2.x; o[9] = r.r2.y; o[10] = r.r2.z;
  o[11] = (float)count[i];
}

__global__ void debug_keys_kernel(const uint32_t* __restrict__ pkey, const uint32_t* __restrict__ pval,
                                  const float* __restrict__ depth, const odgs_status* __restrict__ status, int64_t cap,
                                  int64_t n, uint64_t* __restrict__ keys, uint32_t* __restrict__ gauss) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t m = min((int64_t)status->n_pairs_stored, cap);
  if (j >= m) return;
  const uint32_t item = pval[j];
  keys[j] = ((uint64_t)pkey[j] << 32) | (uint64_t)__float_as_uint(depth[item]);
  gauss[j] = (uint32_t)(item % n);
}

// Coarse binning: the 16x16 tiles' lists sit in the item buffer in four regions (by quadrant of the
// 32x32 tile); written out in global 16x16 tile order (one workgroup: a scan of the list lengths per
// 1024 tiles, then each wavefront copies whole lists).
__global__ __launch_bounds__(1024) void debug_keys_coarse_kernel(const uint2* __restrict__ ranges, int tiles,
                                                                 const uint32_t* __restrict__ items,
                                                                 const float* __restrict__ depth, int64_t cap,
                                                                 int64_t n, uint64_t* __restrict__ keys,
                                                                 uint32_t* __restrict__ gauss) {
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t s_off[1024];
  __shared__ uint2 s_rg[1024];
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t >> 6;
  int64_t carry = 0;
  for (int base = 0; base < tiles; base += 1024) {
    const uint2 rg = base + t < tiles ? ranges[base + t] : make_uint2(0u, 0u);
    const uint32_t len = rg.y - rg.x;
    uint32_t incl = len;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    if (lane == kWave - 1) wsum[w] = incl;
    __syncthreads();
    uint32_t pre = 0, total = 0;
    for (int q = 0; q < 1024 / kWave; ++q) {
      pre += q < w ? wsum[q] : 0u;
      total += wsum[q];
    }
    s_off[t] = pre + incl - len;
    s_rg[t] = rg;
    __syncthreads();
    for (int k = w; k < 1024 && base + k < tiles; k += 1024 / kWave) {
      const uint2 r = s_rg[k];
      const int64_t o = carry + s_off[k];
      for (uint32_t j = lane; j < r.y - r.x; j += kWave) {
        const int64_t pos = o + j;
        if (pos < cap) {
          const uint32_t item = items[r.x + j];
          keys[pos] = ((uint64_t)(base + k) << 32) | (uint64_t)__float_as_uint(depth[item]);
          gauss[pos] = (uint32_t)(item % n);
        }
      }
    }
    carry += total;
    __syncthreads();
  }
}

__global__ void debug_pixel_counts_kernel(const int32_t* __restrict__ last, const int32_t* __restrict__ nc,
                                          const int32_t* __restrict__ ne, const int32_t* __restrict__ le,
                                          int64_t pixels, int32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= pixels) return;
  out[4 * i] = last[i];
  out[4 * i + 1] = nc[i];
  out[4 * i + 2] = ne[i];
  out[4 * i + 3] = le[i];
}

template <int TILE, int BATCH>
struct FwdRun {
  static void run(const odgs_plan* p, const TileSched& sc, const ViewTable& vt, const uint2* ranges,
                  const uint32_t* items, const Rec* rec, float* out_rgb, float* out_T, float* wT, int32_t* wl,
                  int32_t* wn, int32_t* we, int32_t* wle, const float* depth, float* out_depth, uint8_t* qmask,
                  hipStream_t st) {
    const bool count = (p->s.flags & ODGS_FLAG_COUNT_WORK) != 0;
#define ODGS_FWD1(C, D)                                                                                             \
  launch_sched(render_fwd_kernel<TILE, BATCH, C, D>, sc, TILE * TILE, st, vt, ranges, items, rec, out_rgb, out_T, wT, \
               wl, wn, we, wle, p->s.bg[0], p->s.bg[1], p->s.bg[2], depth, out_depth, qmask,                         \
               (int64_t)p->pair_capacity)
    // the counting and depth variants keep one pixel per lane (counters per 8x8 quadrant)
    if (count && out_depth)
      ODGS_FWD1(true, true);
    else if (count)
      ODGS_FWD1(true, false);
    else if (out_depth)
      ODGS_FWD1(false, true);
    else if constexpr (TILE == 16)
      launch_sched(render_fwd4_kernel<16, BATCH>, with_split(sc), kWave, st, vt, ranges, items, rec, out_rgb, out_T,
                   wT, wl, p->s.bg[0], p->s.bg[1], p->s.bg[2], qmask, (int64_t)p->pair_capacity);
    else if constexpr (TILE == 32)
      launch_sched(render_fwd4_kernel<32, BATCH>, with_parts(sc), kWave, st, vt, ranges, items, rec, out_rgb, out_T,
                   wT, wl, p->s.bg[0], p->s.bg[1], p->s.bg[2], qmask, (int64_t)p->pair_capacity);
    else
      ODGS_FWD1(false, false);
#undef ODGS_FWD1
  }
};

template <int TILE, int BATCH>
struct BwdRun {
  static void run(const odgs_plan* p, const TileSched& sc, const ViewTable& vt, const uint2* ranges,
                  const uint32_t* items, const Rec* rec, const float* wT, const int32_t* wl, const float* dL, double* g2d,
                  const uint8_t* qmask, hipStream_t st) {
    // four pixels per lane in one wavefront per 16x16 block (split tiles as the forward split
    // them; 32x32 tiles as four blocks); an 8x8 tile has a single quadrant and keeps one pixel per
    // lane
    if constexpr (TILE == 16)
      launch_sched(render_bwd4_kernel<16, BATCH>, with_split(sc), kWave, st, vt, ranges, items, rec, wT, wl, dL, g2d,
                   p->items, p->s.bg[0], p->s.bg[1], p->s.bg[2], qmask, (int64_t)p->pair_capacity);
    else if constexpr (TILE == 32)
      launch_sched(render_bwd4_kernel<32, BATCH>, with_parts(sc), kWave, st, vt, ranges, items, rec, wT, wl, dL, g2d,
                   p->items, p->s.bg[0], p->s.bg[1], p->s.bg[2], qmask, (int64_t)p->pair_capacity);
    else
      launch_sched(render_bwd_kernel<TILE, BATCH>, sc, TILE * TILE, st, vt, ranges, items, rec, wT, wl, dL, g2d,
                   p->items, p->s.bg[0], p->s.bg[1], p->s.bg[2], qmask);
  }
};

// Dispatch over the supported (tile, batch) pairs; returns false for an unsupported pair.
template <template <int, int> class F, typename... Args>
bool dispatch(int tile, int batch, Args&&... args) {
#define ODGS_CASE(TT, BB)                        \
  if (tile == TT && batch == BB) {               \
    F<TT, BB>::run(std::forward<Args>(args)...); \
    return true;                                 \
  }
  ODGS_CASE(8, 32) ODGS_CASE(8, 64) ODGS_CASE(8, 128) ODGS_CASE(8, 256)
  ODGS_CASE(16, 32) ODGS_CASE(16, 64) ODGS_CASE(16, 128) ODGS_CASE(16, 256)
  ODGS_CASE(32, 64) ODGS_CASE(32, 128) ODGS_CASE(32, 256)
#undef ODGS_CASE
  return false;
}

}  // namespace

hipError_t launch_render_fwd(const odgs_plan* p, void* ws, float* out_rgb, float* out_T, float* out_depth,
                             hipStream_t st) {
  const ViewTable vt = make_view_table(p);
  const int tiles = p->tile_base[p->n_views];
  if (tiles == 0) return hipSuccess;
  const uint2* ranges = ws_ptr<uint2>(ws, p->off_ranges);
  const uint32_t* items = ws_ptr<uint32_t>(ws, p->off_pval[p->pair_final]);
  const Rec* rec = ws_ptr<Rec>(ws, p->off_rec);
  float* wT = ws_ptr<float>(ws, p->off_T);
  int32_t* wl = ws_ptr<int32_t>(ws, p->off_last);
  int32_t* wn = ws_ptr<int32_t>(ws, p->off_ncontrib);
  int32_t* we = ws_ptr<int32_t>(ws, p->off_neval);
  int32_t* wle = ws_ptr<int32_t>(ws, p->off_lasteval);
  const float* depth = ws_ptr<float>(ws, p->off_depth);
  uint8_t* qmask = ws_ptr<uint8_t>(ws, p->off_pval[p->pair_final ^ 1]);  // unused by the sort's result
  const TileSched sc = make_sched(p, ws, 0);
  if (!dispatch<FwdRun>(p->s.tile, p->s.batch, p, sc, vt, ranges, items, rec, out_rgb, out_T, wT, wl, wn, we, wle,
                        depth, out_depth, qmask, st))
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_render_bwd(const odgs_plan* p, void* ws, const float* dL_drgb, hipStream_t st) {
  const ViewTable vt = make_view_table(p);
  const int tiles = p->tile_base[p->n_views];
  if (tiles == 0) return hipSuccess;
  double* g2d = ws_ptr<double>(ws, p->off_g2d);
  const uint2* ranges = ws_ptr<uint2>(ws, p->off_ranges);
  const uint32_t* items = ws_ptr<uint32_t>(ws, p->off_pval[p->pair_final]);
  const Rec* rec = ws_ptr<Rec>(ws, p->off_rec);
  const float* wT = ws_ptr<float>(ws, p->off_T);
  const int32_t* wl = ws_ptr<int32_t>(ws, p->off_last);
  const uint8_t* qmask = ws_ptr<uint8_t>(ws, p->off_pval[p->pair_final ^ 1]);  // written by the forward
  const TileSched sc = make_sched(p, ws, 1);
  if (!dispatch<BwdRun>(p->s.tile, p->s.batch_bwd, p, sc, vt, ranges, items, rec, wT, wl, dL_drgb, g2d, qmask, st))
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_debug_records(const odgs_plan* p, const void* ws, float* out, hipStream_t st) {
  if (p->items == 0) return hipSuccess;
  hipLaunchKernelGGL(debug_records_kernel, dim3((unsigned)((p->items + 255) / 256)), dim3(256), 0, st,
                     ws_ptr<Rec>(ws, p->off_rec), ws_ptr<float>(ws, p->off_depth), ws_ptr<uint32_t>(ws, p->off_count),
                     p->items, out);
  return hipGetLastError();
}

__global__ void debug_copy_kernel(const double* __restrict__ src, int64_t n, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_debug_g2d(const odgs_plan* p, const void* ws, double* out, hipStream_t st) {
  const int64_t n = (int64_t)p->g2d_stride * p->items;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(debug_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     ws_ptr<double>(ws, p->off_g2d), n, out);
  return hipGetLastError();
}

hipError_t launch_debug_pixel_counts(const odgs_plan* p, const void* ws, int32_t* out, hipStream_t st) {
  const int64_t pixels = p->pix_base[p->n_views];
  if (pixels == 0) return hipSuccess;
  hipLaunchKernelGGL(debug_pixel_counts_kernel, dim3((unsigned)((pixels + 255) / 256)), dim3(256), 0, st,
                     ws_ptr<int32_t>(ws, p->off_last), ws_ptr<int32_t>(ws, p->off_ncontrib),
                     ws_ptr<int32_t>(ws, p->off_neval), ws_ptr<int32_t>(ws, p->off_lasteval), pixels, out);
  return hipGetLastError();
}

hipError_t launch_debug_keys(const odgs_plan* p, const void* ws, int64_t cap, uint64_t* keys, uint32_t* gauss,
                             hipStream_t st) {
  if (cap <= 0) return hipSuccess;
  if (p->coarse) {
    hipLaunchKernelGGL(debug_keys_coarse_kernel, dim3(1), dim3(1024), 0, st, ws_ptr<uint2>(ws, p->off_ranges),
                       p->tile_base[p->n_views], ws_ptr<uint32_t>(ws, p->off_pval[p->pair_final]),
                       ws_ptr<float>(ws, p->off_depth), cap, p->n, keys, gauss);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(debug_keys_kernel, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, st,
                     ws_ptr<uint32_t>(ws, p->off_pkey[p->pair_final]), ws_ptr<uint32_t>(ws, p->off_pval[p->pair_final]),
                     ws_ptr<float>(ws, p->off_depth), ws_ptr<odgs_status>(ws, p->off_status), cap, p->n, keys, gauss);
  return hipGetLastError();
}

}  // namespace odgs
