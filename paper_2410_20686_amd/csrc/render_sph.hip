// Compositing kernels of the spherical footprint (ODGS_FLAG_SPHERICAL), gfx950.
//
// Same structure as the affine compositors: at 16x16 tiles one wavefront per tile (or per
// quadrant of a split tile) with four pixels per lane; at 8x8 and 32x32 one workgroup per (view,
// tile), one thread per pixel, every 64-wide wavefront owning an 8x8 quadrant; the tile's
// depth-ordered list is staged through LDS in batches.  What changes is the evaluation: each pixel carries the unit direction
// d of its ray (from the per-view ray table, rounded once to float), and a Gaussian's exponent is
// -qh / D with t1 = u1 . d, t2 = u2 . d, h = w . d, qh = t1^2 + t2^2, D = h^2 + k2 qh (the maximum
// of the 3D Gaussian along the ray, see SphRec); it reaches the pixel iff h > 0 and
// p_min D + qh <= 0.  While the forward stages, a record's quadrant mask comes from its culling
// data (SphCull): a quadrant is skipped when the angle between its centre ray and mu^ exceeds the
// cone half-angle beta plus the quadrant's angular radius, or when the disk that holds the
// gnomonic images of the quadrant's rays misses the item's gnomonic ellipse.  The forward stores
// the masks per list position; the backward loads them.
//
// Backward: per accepted (Gaussian, wavefront) the 13 gradient values (mu^ (3), Sigma~ (6),
// opacity, rgb), summed first over a lane's pixels, are summed over each 16-lane row by a DPP
// butterfly and over rows by the row-swap permutes, kept per wavefront in LDS, and flushed with one
// double atomic per (Gaussian, tile or task, value) to contiguous 104-byte records.
#include "common.h"
#include "wave.h"

#include <utility>

namespace odgs {
namespace {

constexpr float kAlphaMax = 0.99f;
constexpr float kTStop = 1e-4f;
constexpr int kNV = 13;  // gradient values per item

template <int TILE, int BATCH>
struct SphStage {
  static constexpr int N = TILE * TILE;
  static constexpr int NQ = (TILE / 8) * (TILE / 8);
  static constexpr int NW = N / kWave;
  float4 s0[BATCH];
  float4 s1[BATCH];
  float4 s2[BATCH];
  float4 s3[BATCH];
  uint32_t sid[BATCH];
  float dep[BATCH];
  uint8_t list[NQ][BATCH];
  uint32_t wcnt[NW][NQ];
  uint32_t tot[NQ];
  float3 qdir[NQ];  // centre ray of each quadrant
};

// Unit ray direction of pixel (x, y) of view v: (cos theta sin phi, -sin theta, cos theta cos phi),
// each component a double product rounded once to float.
__device__ inline float3 pixel_ray(const double2* __restrict__ dirs, const ViewTable& vt, int v, int x, int y) {
  const double2 c = dirs[vt.dir_base[v] + x];             // (sin phi, cos phi)
  const double2 r = dirs[vt.dir_base[v] + vt.W[v] + y];   // (sin theta, cos theta)
  return make_float3((float)(r.y * c.x), (float)(-r.x), (float)(r.y * c.y));
}

// Angular radius about a quadrant's centre ray (pixel (4, 4) of the 8x8 block) that holds every
// pixel ray of the quadrant: at most 4 pixel pitches in each direction, i.e. 4 pi / H in
// elevation plus 4 (2 pi / W) cos(theta) <= 8 pi / W along the parallel (the path along the
// meridian then the parallel is no shorter than the great circle).
__device__ inline float quadrant_radius(int W, int H) {
  return (4.0f * 3.14159265f / (float)H + 8.0f * 3.14159265f / (float)W) * 1.001f + 1e-6f;
}

template <int TILE, int BATCH>
__device__ inline void sph_stage_init(SphStage<TILE, BATCH>& S, const double2* __restrict__ dirs, const ViewTable& vt,
                                      int v, int tx0, int ty0) {
  constexpr int QPR = TILE / 8;
  if (threadIdx.x < SphStage<TILE, BATCH>::NQ) {
    const int q = threadIdx.x;
    S.qdir[q] = pixel_ray(dirs, vt, v, tx0 + (q % QPR) * 8 + 4, ty0 + (q / QPR) * 8 + 4);
  }
  __syncthreads();
}

// Quadrants of a tile (centre rays qdir[NQ]) that the item's culling data admits, among those in
// `sel` (uniform).  A quadrant is kept unless the angle between its centre ray and mu^ exceeds
// the cone half-angle beta plus the quadrant's angular radius qrad, or the disk that holds the
// gnomonic images of the quadrant's rays misses the item's gnomonic ellipse.
template <int NQ>
__device__ inline uint32_t sph_quadrant_mask(const SphCull& cu, const float3* qdir, float qrad, uint32_t sel = ~0u) {
  const float4 c = cu.c0;
  // cone: hit iff angle(quadrant centre, mu^) <= beta + qrad; the 1e-5 slack covers the float
  // rounding of the dot product and of the cosine
  const float lim = c.w + qrad >= 3.14159f ? -2.0f : cosf(c.w + qrad) - 1e-5f;
  const float cq = cosf(qrad), sq = sinf(qrad);
  uint32_t m = 0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (!((sel >> q) & 1u)) continue;
    const float3 d = qdir[q];
    const float sd = fmaf(d.z, c.z, fmaf(d.y, c.y, d.x * c.x));  // cos of the centre's angle to mu^
    bool hit = sd >= lim;
    // ellipse: every ray of the quadrant is within qrad of the centre ray, hence at most
    // gamma_max = gamma_c + qrad from mu^, and the gnomonic map stretches distances by at most
    // sec^2(gamma_max) there: the images lie within r_q = qrad sec^2(gamma_max) of the
    // centre's image p_c.  The quadrant is kept iff that disk can meet the ellipse:
    // (p_c - p0)^T M (p_c - p0) <= (rho + sqrt(lambda_max) r_q)^2 (1e-3 relative slack).
    const float cmax = fmaf(sd, cq, -sqrtf(fmaxf(0.0f, fmaf(-sd, sd, 1.0f))) * sq);  // cos(gamma_max)
    if (hit && cu.c3.z > 0.0f && cmax > 0.05f) {
      const float inv = 1.0f / sd;
      const float px = fmaf(d.z, cu.c1.y, d.x * cu.c1.x) * inv - cu.c2.y;
      const float py = fmaf(d.z, cu.c2.x, fmaf(d.y, cu.c1.w, d.x * cu.c1.z)) * inv - cu.c2.z;
      const float qv = fmaf(cu.c2.w * px, px, py * fmaf(2.0f * cu.c3.x, px, cu.c3.y * py));
      const float rr = fmaf(cu.c3.w, qrad / (cmax * cmax), cu.c3.z);
      hit = qv <= rr * rr * 1.001f + 1e-6f;
    }
    m |= hit ? (1u << q) : 0u;
  }
  return m;
}

// How the quadrant masks are obtained: evaluated (the forward, which after walking each batch
// stores per list position the quadrants its pixels reached, into the pair buffer the sort leaves
// unused), or loaded from there (the backward, which visits only list positions before its tile's
// last contributor, all staged by the forward).
enum SphMaskMode { kSphMaskEval = 0, kSphMaskLoad = 2 };

// Stage `cnt` records (entry e <- list position first + dir * e) and build every wavefront's
// order-preserving list of the entries whose cone reaches its quadrant.
template <int TILE, int BATCH, int QM = kSphMaskEval>
__device__ inline void sph_stage_batch(SphStage<TILE, BATCH>& S, const uint32_t* __restrict__ pair_items,
                                       const SphRec* __restrict__ rec, const SphCull* __restrict__ cull,
                                       uint32_t first, int dir, int cnt, float qrad,
                                       int (&nq)[SphStage<TILE, BATCH>::NQ], const float* __restrict__ depth,
                                       const uint16_t* __restrict__ qmask_in = nullptr) {
  static_assert(SphStage<TILE, BATCH>::NQ <= 16, "a quadrant mask fits 16 bits");
  using St = SphStage<TILE, BATCH>;
  const int t = threadIdx.x, ln = t & (kWave - 1), wv = t >> 6;
  const uint64_t below = ln == 0 ? 0ull : (~0ull >> (kWave - ln));
#pragma unroll
  for (int q = 0; q < St::NQ; ++q) nq[q] = 0;
  for (int r0 = 0; r0 < cnt; r0 += St::N) {
    const int e = r0 + t;
    uint32_t m = 0;
    if (e < cnt) {
      const uint32_t pos = first + dir * e;
      const uint32_t item = pair_items[pos];
      const SphRec r = rec[item];
      S.s0[e] = r.s0;
      S.s1[e] = r.s1;
      S.s2[e] = r.s2;
      S.s3[e] = r.s3;
      S.sid[e] = item;
      if (depth) S.dep[e] = depth[item];
      if constexpr (QM == kSphMaskLoad) {
        m = qmask_in[pos];
      } else {
        m = sph_quadrant_mask<St::NQ>(cull[item], S.qdir, qrad);
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
    __syncthreads();
  }
}

// Float evaluation of one record for ray d: returns the acceptance; power = -qh / D (correctly
// rounded division); also hands out t1, t2, h, D and qh for the backward.
__device__ inline bool sph_eval(const float4& a, const float4& b, const float4& c, const float3& d, float& power,
                                float& t1, float& t2, float& h, float& D, float& qh) {
  t1 = fmaf(a.z, d.z, fmaf(a.y, d.y, a.x * d.x));
  t2 = fmaf(b.y, d.z, fmaf(b.x, d.y, a.w * d.x));
  h = fmaf(c.x, d.z, fmaf(b.w, d.y, b.z * d.x));
  qh = fmaf(t1, t1, t2 * t2);
  D = fmaf(c.y, qh, h * h);
  power = -__fdiv_rn(qh, D);
  return h > 0.0f && !(fmaf(c.w, D, qh) > 0.0f);
}

template <int TILE, int BATCH, bool DEPTH>
__global__ __launch_bounds__(TILE* TILE) void render_sph_fwd_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items,
    const SphRec* __restrict__ rec, const SphCull* __restrict__ cull, const double2* __restrict__ dirs,
    float* __restrict__ out_rgb, float* __restrict__ out_T, float* __restrict__ ws_T, int32_t* __restrict__ ws_last,
    float bg0, float bg1, float bg2, const float* __restrict__ depth, float* __restrict__ out_depth,
    uint16_t* __restrict__ qmask, TileSched sc) {
  using St = SphStage<TILE, BATCH>;
  constexpr int N = St::N;
  __shared__ St S;
  // s_used[q][e]: some still-compositing pixel of quadrant q reaches entry e of the batch being
  // walked (before a pixel's last contributor this test and the backward's are the same float
  // decision); after the batch these quadrants are the mask handed to the backward
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
    const int wq = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const float3 d = pixel_ray(dirs, vt, v, x, y);
    const float qrad = quadrant_radius(W, H);
    sph_stage_init<TILE, BATCH>(S, dirs, vt, v, tx0, ty0);
    const uint2 rg = ranges[g];
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, Dsum = 0.0f;
    int last = 0;
    int done = 0;  // an int rather than a bool: the ballots below then compile to one compare
    // writes the masks of the batch walked last (after a barrier) and clears s_used for the next
    auto flush_used = [&](uint32_t first, int n_walked) {
      for (int e = threadIdx.x; e < BATCH; e += N) {
        if (e < n_walked) {
          uint32_t mq = 0;
#pragma unroll
          for (int q = 0; q < St::NQ; ++q) mq |= s_used[q][e] ? (1u << q) : 0u;
          qmask[first + e] = (uint16_t)mq;
        }
#pragma unroll
        for (int q = 0; q < St::NQ; ++q) s_used[q][e] = 0;
      }
    };
    uint32_t walked_base = 0;
    int walked_cnt = 0;
    for (uint32_t base = rg.x; base < rg.y; base += BATCH) {
      const bool all_done = __syncthreads_count(done) == N;
      flush_used(walked_base, walked_cnt);
      walked_cnt = 0;
      if (all_done) break;
      const int cnt = (int)min((uint32_t)BATCH, rg.y - base);
      int nq[St::NQ];
      sph_stage_batch<TILE, BATCH>(S, pair_items, rec, cull, base, 1, cnt, qrad, nq, DEPTH ? depth : nullptr);
      const int n = __builtin_amdgcn_readfirstlane(nq[wq]);
      for (int i = 0; i < n; ++i) {
        if (__builtin_amdgcn_ballot_w64(done == 0) == 0ull) break;  // uniform: every pixel has finished
        const int k = S.list[wq][i];
        const float4 c = S.s2[k];
        float power, t1, t2, h, D, qh;
        const bool hit = sph_eval(S.s0[k], S.s1[k], c, d, power, t1, t2, h, D, qh);
        const bool ok = done == 0 && hit;
        if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
        s_used[wq][k] = 1;  // reached here (accepted unless that pixel stops at it: a superset)
        const float alpha = fminf(c.z * __expf(power), kAlphaMax);
        const float Tn = T * (1.0f - alpha);
        const bool acc = ok && !(Tn < kTStop);
        done = ok != acc ? 1 : done;  // stop: reached, but T would drop below 1e-4
        const float4 col = S.s3[k];
        const float w = acc ? alpha * T : 0.0f;
        C0 = fmaf(w, col.x, C0);
        C1 = fmaf(w, col.y, C1);
        C2 = fmaf(w, col.z, C2);
        if (DEPTH) Dsum = Dsum + w * S.dep[k];
        T = acc ? Tn : T;
        last = acc ? (int)(base - rg.x) + k + 1 : last;
      }
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
    if (DEPTH) out_depth[gp] = Dsum;
    if (out_T) out_T[gp] = T;
  }
}

// Sums thirteen per-lane values over each 16-lane row in four DPP exchange steps (partners
// 15 - i, 7 - i, 3 - i, i ^ 1 inside the row).  Each step pairs the registers a lane holds, the lane
// keeping one slot of each pair by a bit of its index, except that values 5, 6 and 7 (which have
// no partner slot) are summed in place in the first step.  Lane i ends with the row sum of value
// kSphRowSlot[i % 16] (none where the table says 15: the second copies of values 5, 6, 7).
constexpr uint64_t kSphRowSlot = 0xFBF9FAC873516240ull;  // nibble i = value index held by row lane i

__device__ inline float row_reduce13(const float (&g)[kNV], int lane) {
#pragma clang fp contract(off)  // keeps the in-place sums single DPP adds (not an FMA with the product)
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2, b0 = lane & 1;
  float a[8];
#pragma unroll
  for (int j = 0; j < 5; ++j) a[j] = bfly<0x140>(g[j], g[8 + j], b3);  // row_mirror
#pragma unroll
  for (int j = 5; j < 8; ++j) a[j] = g[j] + dpp_read<0x140>(g[j]);
  float c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) c[j] = bfly<0x141>(a[2 * j], a[2 * j + 1], b2);  // row_half_mirror
  const float e0 = bfly<0x1B>(c[0], c[1], b1);                                 // quad_perm [3,2,1,0]
  const float e1 = bfly<0x1B>(c[2], c[3], b1);
  return bfly<0xB1>(e0, e1, b0);                                               // quad_perm [1,0,3,2]
}

// g2d layout [items][13]: d/dmu^ (3), d/dSigma~ (xx, xy, xz, yy, yz, zz; off-diagonals as one
// shared variable), d/dopacity, d/d(r, g, b).  With A = Sigma~^-1 and the ray's closest approach
// t* d (t* = h / D) the exponent p = -m / 2 has dp/dmu^ = z and dp/dSigma~ = z z^T / 2, where
// z = A (t* d - mu^) = 2 N^T y, y = (h t1, h t2, qh) / D, N = [u1; u2; -w] (rows; A = 2 (u1 u1^T +
// u2 u2^T) + (2 / k2) w w^T, u1, u2 tangent, w . mu^ = 1).  y is the offset in the Gaussian's
// whitened coordinates (up to constant factors per component), all three of the same order, so the
// per-tile sums S_y = sum dpow y and Y = sum dpow y y^T stay well scaled for any shape; they map
// exactly to g_mu^ = 2 N^T S_y and g_Sigma~ = 2 N^T Y N, applied once per (Gaussian, tile) in
// double at the flush.
template <int NS, int B>
__device__ inline double sph_acc_total(const float (&acc)[NS][kNV][B], int q, int t) {
  double s = (double)acc[0][q][t];
#pragma unroll
  for (int w = 1; w < NS; ++w) s += (double)acc[w][q][t];
  return s;
}

// Component i of the columns of N = [u1; u2; -w] (rows), i.e. (u1_i, u2_i, -w_i), from the staged
// record words (u1 = a.xyz, u2 = (a.w, b.x, b.y), w = (b.z, b.w, c.x)); selects, no indexed array.
__device__ inline void sph_ncol(int i, const float4& a, const float4& b, const float4& c, float& n0, float& n1,
                                float& n2) {
  n0 = i == 0 ? a.x : (i == 1 ? a.y : a.z);
  n1 = i == 0 ? a.w : (i == 1 ? b.x : b.y);
  n2 = -(i == 0 ? b.z : (i == 1 ? b.w : c.x));
}

// Value q of an entry's gradient record (layout of g2d) from its per-wavefront sums (slots: S_y (3),
// Y (y1y1, y1y2, y1y3, y2y2, y2y3, y3y3), opacity, rgb); a, b, c: the entry's staged record words.
template <int NS, int B>
__device__ inline double sph_flush_value(const float (&acc)[NS][kNV][B], int q, int t, const float4& a, const float4& b,
                                         const float4& c) {
  if (q >= 9) return sph_acc_total(acc, q, t);
  if (q < 3) {
    float n0, n1, n2;
    sph_ncol(q, a, b, c, n0, n1, n2);
    return 2.0 * ((double)n0 * sph_acc_total(acc, 0, t) + (double)n1 * sph_acc_total(acc, 1, t) +
                  (double)n2 * sph_acc_total(acc, 2, t));
  }
  // Sigma~ entry (i, j), q - 3 = 0..5 -> (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
  const int i = (q >= 6) + (q >= 8), j = q == 3 ? 0 : ((q == 4 || q == 6) ? 1 : 2);
  float a0, a1, a2, b0, b1, b2;
  sph_ncol(i, a, b, c, a0, a1, a2);
  sph_ncol(j, a, b, c, b0, b1, b2);
  const double y00 = sph_acc_total(acc, 3, t), y01 = sph_acc_total(acc, 4, t), y02 = sph_acc_total(acc, 5, t);
  const double y11 = sph_acc_total(acc, 6, t), y12 = sph_acc_total(acc, 7, t), y22 = sph_acc_total(acc, 8, t);
  // n_i^T Y n_j
  const double m0 = y00 * b0 + y01 * b1 + y02 * b2;
  const double m1 = y01 * b0 + y11 * b1 + y12 * b2;
  const double m2 = y02 * b0 + y12 * b1 + y22 * b2;
  const double nyn = a0 * m0 + a1 * m1 + a2 * m2;
  return (i == j ? 2.0 : 4.0) * nyn;  // the shared off-diagonal takes both symmetric entries
}

// One pixel per lane (tiles of 8 and 32).
template <int TILE, int BATCH>
__global__ __launch_bounds__(TILE* TILE) void render_sph_bwd_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items,
    const SphRec* __restrict__ rec, const SphCull* __restrict__ cull, const double2* __restrict__ dirs,
    const float* __restrict__ ws_T, const int32_t* __restrict__ ws_last, const float* __restrict__ dL_drgb,
    double* __restrict__ g2d, float bg0, float bg1, float bg2, const uint16_t* __restrict__ qmask, TileSched sc) {
  using St = SphStage<TILE, BATCH>;
  constexpr int N = St::N;
  // A slot set per wavefront up to four wavefronts; beyond (tile 32: sixteen) wavefronts w and
  // w + NW / 2 share set w % (NW / 2) and add into it: two additions onto a cleared slot give the
  // same float in either order, so the per-tile sums do not depend on wavefront timing.
  constexpr int NS = St::NW <= 4 ? St::NW : St::NW / 2;
  __shared__ St S;
  __shared__ float acc[NS][kNV][BATCH + 1];
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
    const float3 d = pixel_ray(dirs, vt, v, x, y);
    const float qrad = quadrant_radius(W, H);
    sph_stage_init<TILE, BATCH>(S, dirs, vt, v, tx0, ty0);
    const uint2 rg = ranges[g];
    const int64_t plane = (int64_t)W * H;
    const int64_t pix = (int64_t)y * W + x;
    const int64_t gp = vt.pix_base[v] + pix;
    const float* dimg = dL_drgb + 3 * vt.pix_base[v];
    const float dl0 = dimg[pix], dl1 = dimg[plane + pix], dl2 = dimg[2 * plane + pix];
    float T = ws_T[gp];
    const int last = ws_last[gp];
    // dL/dC . (colour of everything behind, incl. background), one scalar for the three channels
    float DS = T * fmaf(dl0, bg0, fmaf(dl1, bg1, dl2 * bg2));
    int wmax = last;
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
          for (int q = 0; q < kNV; ++q) acc[w][q][t] = 0.0f;
      }
      int nq[St::NQ];
      // entry e is list position end - 1 - e (back to front)
      sph_stage_batch<TILE, BATCH, kSphMaskLoad>(S, pair_items, rec, cull, rg.x + end - 1, -1, cnt, qrad, nq, nullptr,
                                                 qmask);
      const int n = __builtin_amdgcn_readfirstlane(nq[wq]);
      for (int i = 0; i < n; ++i) {
        const int k = __builtin_amdgcn_readfirstlane(S.list[wq][i]);
        const int jrel = end - 1 - k;
        if (jrel >= wmax) continue;  // uniform: behind every contributor of this wavefront
        const float4 a = S.s0[k], b = S.s1[k], c = S.s2[k];
        float power, t1, t2, h, D, qh;
        // evaluated on every lane (no short circuit): the gradient terms below are formed on all
        // lanes and zeroed by selects, which needs finite operands
        const bool hit = sph_eval(a, b, c, d, power, t1, t2, h, D, qh);
        const bool ok = jrel < last && hit;
        if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
        const float G = __expf(power);
        const float araw = c.z * G;
        const bool live = ok && !(araw > kAlphaMax);  // contributes and unclamped
        // alpha = 0 where the Gaussian does not contribute, so its weight below is 0 without a select
        const float alpha = ok ? fminf(araw, kAlphaMax) : 0.0f;
        const float inv_om = __builtin_amdgcn_rcpf(1.0f - alpha);
        T = T * inv_om;  // transmittance in front of this Gaussian (alpha = 0: times exactly 1)
        const float wk = alpha * T;
        const float4 col = S.s3[k];
        const float dc = fmaf(dl0, col.x, fmaf(dl1, col.y, dl2 * col.z));  // dL/dC . colour
        const float dL_da = fmaf(dc, T, -DS * inv_om);
        DS = fmaf(dc, wk, DS);
        const float dla = live ? dL_da : 0.0f;
        const float dpow = dla * alpha;
        // whitened offset y = (h t1, h t2, qh) / D, zero on lanes that do not contribute (D may be
        // 0 there)
        const float s1 = live ? __builtin_amdgcn_rcpf(D) : 0.0f;
        const float y1 = s1 * (h * t1), y2 = s1 * (h * t2), y3 = s1 * qh;
        const float gx = dpow * y1, gy = dpow * y2, gz = dpow * y3;
        const float gv[kNV] = {gx,      gy,      gz,       gx * y1,  gx * y2,  gx * y3, gy * y2,
                               gy * y3, gz * y3, dla * G, wk * dl0, wk * dl1, wk * dl2};
        const float rs = row_reduce13(gv, lane);
        const int slot = (int)((kSphRowSlot >> (4 * (lane & 15))) & 0xF);
        const float ws = sum_rows(rs);
        if (lane < 16 && slot < kNV) {
          if constexpr (St::NW > NS)
            atomicAdd(&acc[wq % NS][slot][k], ws);
          else
            acc[wq][slot][k] = ws;
        }
      }
      __syncthreads();
      // thirteen consecutive lanes carry one entry's values: contiguous 104-byte records
#pragma unroll 1
      for (int xx = threadIdx.x; xx < kNV * cnt; xx += N) {
        const int t = xx / kNV, q = xx - kNV * t;
        const double s = sph_flush_value(acc, q, t, S.s0[t], S.s1[t], S.s2[t]);
        if (s != 0.0) unsafeAtomicAdd(&g2d[(int64_t)S.sid[t] * kNV + q], s);
      }
      __syncthreads();
    }
  }
}

// One-wavefront compositing of a 16x16 tile, four pixels per lane (lane l holds pixel (l % 8, l / 8)
// of each 8x8 quadrant q = 2 qy + qx), as in the affine compositors: the list is staged once per
// batch with each entry's quadrant mask (one 16-bit LDS word, entry | mask << 8), an entry is
// evaluated only for the quadrants in its mask, and the reverse compositor reduces the four
// pixels' 13 gradient values across lanes once per entry.  A task is a whole tile or one quadrant
// of a split tile (TileSched); the culling masks handed from the forward to the backward are one
// byte per list position, in the byte plane of the task's quadrant (plane q at byte offset
// q * qplane; whole tiles use plane 0).
template <int BATCH, bool DEPTH>
struct SphFwdStage4 {
  float4 s0[BATCH];
  float4 s1[BATCH];
  float4 s2[BATCH];
  float4 s3[BATCH];
  float dep[DEPTH ? BATCH : 1];
  uint16_t list[BATCH];
  uint8_t used[BATCH];
  float3 qdir[4];
};

template <int BATCH, bool DEPTH>
__global__ __launch_bounds__(kWave) void render_sph_fwd4_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items,
    const SphRec* __restrict__ rec, const SphCull* __restrict__ cull, const double2* __restrict__ dirs,
    float* __restrict__ out_rgb, float* __restrict__ out_T, float* __restrict__ ws_T, int32_t* __restrict__ ws_last,
    float bg0, float bg1, float bg2, const float* __restrict__ depth, float* __restrict__ out_depth,
    uint8_t* __restrict__ qmask, int64_t qplane, TileSched sc) {
  constexpr int TILE = 16;
  __shared__ SphFwdStage4<BATCH, DEPTH> S;
  const int nsplit = forward_split(sc);
  mark_forward(sc, nsplit);
  __shared__ uint32_t s_claim;
  uint32_t round = 0, sel = 0;
  const int lane = threadIdx.x;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  for (int g; (g = claim_task(sc, nsplit, round, &s_claim, sel)) >= 0;) {
    const int v = view_of_tile(vt, g);
    const int W = vt.W[v], H = vt.H[v];
    const int ntx = W / TILE;
    const int lt = g - vt.tile_base[v];
    const int tx0 = (lt % ntx) * TILE, ty0 = (lt / ntx) * TILE;
    const int x = tx0 + (lane & 7), y = ty0 + (lane >> 3);
    float3 d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) d[q] = pixel_ray(dirs, vt, v, x + 8 * (q & 1), y + 8 * (q >> 1));
    const float qrad = quadrant_radius(W, H);
    if (lane < 4) S.qdir[lane] = pixel_ray(dirs, vt, v, tx0 + (lane & 1) * 8 + 4, ty0 + (lane >> 1) * 8 + 4);
    __syncthreads();
    const uint2 rg = ranges[g];
    float T[4], C0[4], C1[4], C2[4], Ds[4];
    int last[4], done[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      T[q] = 1.0f;
      C0[q] = C1[q] = C2[q] = Ds[q] = 0.0f;
      last[q] = 0;
      done[q] = 0;
    }
    uint32_t alive = sel;  // selected quadrants with a pixel still compositing (uniform)
    uint8_t* qm = qmask + (sel == 0xFu ? 0 : (int64_t)__builtin_ctz(sel) * qplane);
    for (uint32_t base = rg.x; base < rg.y && alive != 0u; base += BATCH) {
      const int cnt = (int)min((uint32_t)BATCH, rg.y - base);
      int n = 0;
      for (int r0 = 0; r0 < cnt; r0 += kWave) {
        const int e = r0 + lane;
        uint32_t m = 0;
        if (e < cnt) {
          const uint32_t item = pair_items[base + e];
          const SphRec r = rec[item];
          S.s0[e] = r.s0;
          S.s1[e] = r.s1;
          S.s2[e] = r.s2;
          S.s3[e] = r.s3;
          if constexpr (DEPTH) S.dep[e] = depth[item];
          S.used[e] = 0;
          m = sph_quadrant_mask<4>(cull[item], S.qdir, qrad, sel);
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
        const float4 a = S.s0[k], b = S.s1[k], c = S.s2[k];
        const float4 col = S.s3[k];  // once per entry, not per accepting quadrant
        uint32_t used = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!((mq >> q) & 1u)) continue;  // uniform
          float power, t1, t2, h, D, qh;
          const bool hit = sph_eval(a, b, c, d[q], power, t1, t2, h, D, qh);
          const bool ok = done[q] == 0 && hit;
          if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
          used |= 1u << q;  // reached here (accepted unless that pixel stops at it: a superset)
          const float alpha = fminf(c.z * __expf(power), kAlphaMax);
          const float Tn = T[q] * (1.0f - alpha);
          const bool acc = ok && !(Tn < kTStop);
          done[q] = ok != acc ? 1 : done[q];  // stop: reached, but T would drop below 1e-4
          const float w = acc ? alpha * T[q] : 0.0f;
          C0[q] = fmaf(w, col.x, C0[q]);
          C1[q] = fmaf(w, col.y, C1[q]);
          C2[q] = fmaf(w, col.z, C2[q]);
          if constexpr (DEPTH) Ds[q] = Ds[q] + w * S.dep[k];
          T[q] = acc ? Tn : T[q];
          last[q] = acc ? (int)(base - rg.x) + k + 1 : last[q];
        }
        if (lane == 0 && used) S.used[k] = (uint8_t)used;
      }
      // quadrants whose pixels have all stopped, taken once per batch
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (((alive >> q) & 1u) && __builtin_amdgcn_ballot_w64(done[q] == 0) == 0ull) alive &= ~(1u << q);
      __syncthreads();
      for (int e = lane; e < cnt; e += kWave) qm[base + e] = S.used[e];
      __syncthreads();
    }
    // list positions past the point where every pixel stopped keep no mask: the backward, which
    // stops at each quadrant's last contributor, never reads them
    const int64_t plane = (int64_t)W * H;
    float* img = out_rgb + 3 * vt.pix_base[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((sel >> q) & 1u)) continue;
      const int64_t pix = (int64_t)(y + 8 * (q >> 1)) * W + x + 8 * (q & 1);
      img[pix] = fmaf(T[q], bg0, C0[q]);
      img[plane + pix] = fmaf(T[q], bg1, C1[q]);
      img[2 * plane + pix] = fmaf(T[q], bg2, C2[q]);
      const int64_t gp = vt.pix_base[v] + pix;
      ws_T[gp] = T[q];
      ws_last[gp] = last[q];
      if constexpr (DEPTH) out_depth[gp] = Ds[q];
      if (out_T) out_T[gp] = T[q];
    }
  }
}

template <int BATCH>
struct SphBwdStage4 {
  float4 s0[BATCH];
  float4 s1[BATCH];
  float4 s2[BATCH];
  float4 s3[BATCH];
  uint32_t sid[BATCH];
  uint16_t list[BATCH];
};

template <int BATCH>
__global__ __launch_bounds__(kWave) void render_sph_bwd4_kernel(
    ViewTable vt, const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_items,
    const SphRec* __restrict__ rec, const double2* __restrict__ dirs, const float* __restrict__ ws_T,
    const int32_t* __restrict__ ws_last, const float* __restrict__ dL_drgb, double* __restrict__ g2d, float bg0,
    float bg1, float bg2, const uint8_t* __restrict__ qmask, int64_t qplane, TileSched sc) {
  constexpr int TILE = 16;
  __shared__ SphBwdStage4<BATCH> S;
  __shared__ float acc[1][kNV][BATCH + 1];
  if (forward_is_stale(sc)) return;  // uniform
  const int nsplit = reverse_split(sc);
  __shared__ uint32_t s_claim;
  uint32_t round = 0, sel = 0;
  const int lane = threadIdx.x;
  const int slot = (int)((kSphRowSlot >> (4 * (lane & 15))) & 0xF);
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  for (int g; (g = claim_task(sc, nsplit, round, &s_claim, sel)) >= 0;) {
    const int v = view_of_tile(vt, g);
    const int W = vt.W[v], H = vt.H[v];
    const int ntx = W / TILE;
    const int lt = g - vt.tile_base[v];
    const int tx0 = (lt % ntx) * TILE, ty0 = (lt / ntx) * TILE;
    const int x = tx0 + (lane & 7), y = ty0 + (lane >> 3);
    const uint2 rg = ranges[g];
    const int64_t plane = (int64_t)W * H;
    const float* dimg = dL_drgb + 3 * vt.pix_base[v];
    float3 d[4];
    float dl0[4], dl1[4], dl2[4], T[4], DS[4];
    int last[4], qmax[4];  // qmax: the quadrant's last contributor over its pixels (uniform)
    int wmax = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((sel >> q) & 1u)) {
        last[q] = 0;  // not this task's: never reached, its other members never read
        qmax[q] = 0;
        continue;
      }
      const int px = x + 8 * (q & 1), py = y + 8 * (q >> 1);
      const int64_t pix = (int64_t)py * W + px;
      const int64_t gp = vt.pix_base[v] + pix;
      d[q] = pixel_ray(dirs, vt, v, px, py);
      dl0[q] = dimg[pix], dl1[q] = dimg[plane + pix], dl2[q] = dimg[2 * plane + pix];
      T[q] = ws_T[gp];
      last[q] = ws_last[gp];
      // dL/dC . (colour of everything behind, incl. background), one scalar for the three channels
      DS[q] = T[q] * fmaf(dl0[q], bg0, fmaf(dl1[q], bg1, dl2[q] * bg2));
      int m = last[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off));
      qmax[q] = __builtin_amdgcn_readfirstlane(m);
      wmax = max(wmax, qmax[q]);
    }
    const uint8_t* qm = qmask + (sel == 0xFu ? 0 : (int64_t)__builtin_ctz(sel) * qplane);
    for (int end = wmax; end > 0; end -= BATCH) {
      const int cnt = min(BATCH, end);
      // stage entries end - 1 - e (back to front) with the forward's masks; list those reaching
      // any selected quadrant, in order
      int n = 0;
      for (int r0 = 0; r0 < cnt; r0 += kWave) {
        const int e = r0 + lane;
        uint32_t m = 0;
        if (e < cnt) {
          const uint32_t pos = rg.x + end - 1 - e;
          m = qm[pos] & sel;
          if (m != 0u) {  // records only of the entries the forward's pixels reached
            const uint32_t item = pair_items[pos];
            const SphRec r = rec[item];
            S.s0[e] = r.s0;
            S.s1[e] = r.s1;
            S.s2[e] = r.s2;
            S.s3[e] = r.s3;
            S.sid[e] = item;
#pragma unroll
            for (int j = 0; j < kNV; ++j) acc[0][j][e] = 0.0f;
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
        const uint32_t mq = km >> 8;
        const float4 a = S.s0[k], b = S.s1[k], c = S.s2[k];
        const float4 col = S.s3[k];
        float gv[kNV];
#pragma unroll
        for (int j = 0; j < kNV; ++j) gv[j] = 0.0f;
        bool any = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (!((mq >> q) & 1u) || jrel >= qmax[q]) continue;  // uniform
          float power, t1, t2, h, D, qh;
          // evaluated on every lane (no short circuit): the gradient terms below are formed on
          // all lanes and zeroed by selects, which needs finite operands
          const bool hit = sph_eval(a, b, c, d[q], power, t1, t2, h, D, qh);
          const bool ok = jrel < last[q] && hit;
          if (__builtin_amdgcn_ballot_w64(ok) == 0ull) continue;  // uniform
          any = true;
          const float G = __expf(power);
          const float araw = c.z * G;
          const bool live = ok && !(araw > kAlphaMax);  // contributes and unclamped
          // alpha = 0 where the Gaussian does not contribute, so its weight below is 0 without a select
          const float alpha = ok ? fminf(araw, kAlphaMax) : 0.0f;
          const float inv_om = __builtin_amdgcn_rcpf(1.0f - alpha);
          T[q] = T[q] * inv_om;  // transmittance in front of this Gaussian (alpha = 0: times exactly 1)
          const float wk = alpha * T[q];
          const float dc = fmaf(dl0[q], col.x, fmaf(dl1[q], col.y, dl2[q] * col.z));  // dL/dC . colour
          const float dL_da = fmaf(dc, T[q], -DS[q] * inv_om);
          DS[q] = fmaf(dc, wk, DS[q]);
          const float dla = live ? dL_da : 0.0f;
          const float dpow = dla * alpha;
          // whitened offset y = (h t1, h t2, qh) / D, zero on lanes that do not contribute
          const float s1 = live ? __builtin_amdgcn_rcpf(D) : 0.0f;
          const float y1 = s1 * (h * t1), y2 = s1 * (h * t2), y3 = s1 * qh;
          const float gx = dpow * y1, gy = dpow * y2, gz = dpow * y3;
          gv[0] += gx;
          gv[1] += gy;
          gv[2] += gz;
          gv[3] = fmaf(gx, y1, gv[3]);
          gv[4] = fmaf(gx, y2, gv[4]);
          gv[5] = fmaf(gx, y3, gv[5]);
          gv[6] = fmaf(gy, y2, gv[6]);
          gv[7] = fmaf(gy, y3, gv[7]);
          gv[8] = fmaf(gz, y3, gv[8]);
          gv[9] = fmaf(dla, G, gv[9]);
          gv[10] = fmaf(wk, dl0[q], gv[10]);
          gv[11] = fmaf(wk, dl1[q], gv[11]);
          gv[12] = fmaf(wk, dl2[q], gv[12]);
        }
        if (!any) continue;  // uniform
        const float rs = row_reduce13(gv, lane);
        const float ws = sum_rows(rs);
        if (lane < 16 && slot < kNV) acc[0][slot][k] = ws;
      }
      __syncthreads();
      // thirteen consecutive lanes carry one listed entry's values: contiguous 104-byte records
#pragma unroll 1
      for (int xx = lane; xx < kNV * n; xx += kWave) {
        const int i = xx / kNV, q = xx - kNV * i;
        const int t = S.list[i] & 0xFF;
        const double s = sph_flush_value(acc, q, t, S.s0[t], S.s1[t], S.s2[t]);
        if (s != 0.0) unsafeAtomicAdd(&g2d[(int64_t)S.sid[t] * kNV + q], s);
      }
      __syncthreads();
    }
  }
}

template <int TILE, int BATCH>
struct SphFwdRun {
  static void run(const odgs_plan* p, const TileSched& sc, const ViewTable& vt, const uint2* ranges,
                  const uint32_t* items, const SphRec* rec, const SphCull* cone, const double2* dirs, float* out_rgb,
                  float* out_T, float* wT, int32_t* wl, const float* depth, float* out_depth, void* qmask_buf,
                  hipStream_t st) {
    // masks: bytes in per-quadrant planes at 16x16 (four pixels per lane), 16 bits per position
    // otherwise
    uint16_t* qmask = static_cast<uint16_t*>(qmask_buf);
    uint8_t* qmask8 = static_cast<uint8_t*>(qmask_buf);
    const int64_t qplane = p->pair_capacity;
    if constexpr (TILE == 16) {
      if (out_depth)
        launch_sched(render_sph_fwd4_kernel<BATCH, true>, with_split(sc), kWave, st, vt, ranges, items, rec, cone, dirs,
                     out_rgb, out_T, wT, wl, p->s.bg[0], p->s.bg[1], p->s.bg[2], depth, out_depth, qmask8, qplane);
      else
        launch_sched(render_sph_fwd4_kernel<BATCH, false>, with_split(sc), kWave, st, vt, ranges, items, rec, cone,
                     dirs, out_rgb, out_T, wT, wl, p->s.bg[0], p->s.bg[1], p->s.bg[2], depth, out_depth, qmask8,
                     qplane);
    } else if (out_depth)
      launch_sched(render_sph_fwd_kernel<TILE, BATCH, true>, sc, TILE * TILE, st, vt, ranges, items, rec, cone, dirs,
                   out_rgb, out_T, wT, wl, p->s.bg[0], p->s.bg[1], p->s.bg[2], depth, out_depth, qmask);
    else
      launch_sched(render_sph_fwd_kernel<TILE, BATCH, false>, sc, TILE * TILE, st, vt, ranges, items, rec, cone, dirs,
                   out_rgb, out_T, wT, wl, p->s.bg[0], p->s.bg[1], p->s.bg[2], depth, out_depth, qmask);
  }
};

template <int TILE, int BATCH>
struct SphBwdRun {
  static void run(const odgs_plan* p, const TileSched& sc, const ViewTable& vt, const uint2* ranges,
                  const uint32_t* items, const SphRec* rec, const SphCull* cone, const double2* dirs, const float* wT,
                  const int32_t* wl, const float* dL, double* g2d, const void* qmask_buf, hipStream_t st) {
    if constexpr (TILE == 16)
      launch_sched(render_sph_bwd4_kernel<BATCH>, with_split(sc), kWave, st, vt, ranges, items, rec, dirs, wT, wl, dL,
                   g2d, p->s.bg[0], p->s.bg[1], p->s.bg[2], static_cast<const uint8_t*>(qmask_buf),
                   (int64_t)p->pair_capacity);
    else
      launch_sched(render_sph_bwd_kernel<TILE, BATCH>, sc, TILE * TILE, st, vt, ranges, items, rec, cone, dirs, wT, wl,
                   dL, g2d, p->s.bg[0], p->s.bg[1], p->s.bg[2], static_cast<const uint16_t*>(qmask_buf));
  }
};

template <template <int, int> class F, typename... Args>
bool sph_dispatch(int tile, int batch, Args&&... args) {
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

hipError_t launch_render_sph_fwd(const odgs_plan* p, void* ws, float* out_rgb, float* out_T, float* out_depth,
                                 hipStream_t st) {
  const ViewTable vt = make_view_table(p);
  const int tiles = p->tile_base[p->n_views];
  if (tiles == 0) return hipSuccess;
  if (!sph_dispatch<SphFwdRun>(p->s.tile, p->s.batch, p, make_sched(p, ws, 0), vt, ws_ptr<uint2>(ws, p->off_ranges),
                               ws_ptr<uint32_t>(ws, p->off_pval[p->pair_final]), ws_ptr<SphRec>(ws, p->off_srec),
                               ws_ptr<SphCull>(ws, p->off_cone), ws_ptr<double2>(ws, p->off_dirs), out_rgb, out_T,
                               ws_ptr<float>(ws, p->off_T), ws_ptr<int32_t>(ws, p->off_last),
                               ws_ptr<float>(ws, p->off_depth), out_depth,
                               ws_ptr<void>(ws, p->off_pval[p->pair_final ^ 1]), st))  // masks: unused pair buffer
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_render_sph_bwd(const odgs_plan* p, void* ws, const float* dL_drgb, hipStream_t st) {
  const ViewTable vt = make_view_table(p);
  const int tiles = p->tile_base[p->n_views];
  if (tiles == 0) return hipSuccess;
  if (!sph_dispatch<SphBwdRun>(p->s.tile, p->s.batch_bwd, p, make_sched(p, ws, 1), vt, ws_ptr<uint2>(ws, p->off_ranges),
                               ws_ptr<uint32_t>(ws, p->off_pval[p->pair_final]), ws_ptr<SphRec>(ws, p->off_srec),
                               ws_ptr<SphCull>(ws, p->off_cone), ws_ptr<double2>(ws, p->off_dirs),
                               ws_ptr<float>(ws, p->off_T), ws_ptr<int32_t>(ws, p->off_last), dL_drgb,
                               ws_ptr<double>(ws, p->off_g2d),
                               ws_ptr<const void>(ws, p->off_pval[p->pair_final ^ 1]), st))  // the forward's masks
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace odgs
