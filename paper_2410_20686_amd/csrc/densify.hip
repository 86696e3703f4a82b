// Densification step of ODGS (Sec. 3.3 with the clone / split / prune rules of 3DGS that the
// method keeps): classify every Gaussian from the statistics gathered by the reverse projection
// stage, then write the surviving originals, the clones and the two children of every split
// Gaussian into the output arrays, each group in parent order.
//
// Three launches: per-block counts of the three output groups (wave ballots), one exclusive scan
// of those counts (a single block), and a scatter that recomputes each Gaussian's class and its
// rank inside its block.  Every decision is an FP32 comparison of the inputs, so the result is
// exactly reproducible; the children's positions are computed in FP32.
#include "common.h"

namespace odgs {
namespace {

constexpr int kDensThreads = 256;
constexpr int kDensWaves = kDensThreads / 64;
constexpr int kScanThreads = 1024;

struct DensRule {
  float big;        // percent_dense * extent: clone at or below, split above
  float min_op;     // prune below this opacity
  float max_scale;  // prune a largest scale above this (when > 0)
};

struct Cls {
  bool orig, clone, child;  // surviving original, surviving clone, surviving children (both)
};

__device__ inline Cls classify(int64_t i, int64_t n, const float* __restrict__ scales, const float* __restrict__ opac,
                               const float* __restrict__ grad_sum, const float* __restrict__ tau_sum,
                               const int32_t* __restrict__ count, const DensRule& rule) {
  const float s0 = scales[i], s1 = scales[n + i], s2 = scales[2 * n + i];
  const float op = opac[i];
  const bool sel = count[i] > 0 && grad_sum[i] >= tau_sum[i];
  const float smax = fmaxf(fmaxf(s0, s1), s2);
  const bool clone = sel && smax <= rule.big;
  const bool split = sel && smax > rule.big;
  const float cmax = fmaxf(fmaxf(s0 / 1.6f, s1 / 1.6f), s2 / 1.6f);
  const bool drop = op < rule.min_op || (rule.max_scale > 0.0f && smax > rule.max_scale);
  const bool drop_child = op < rule.min_op || (rule.max_scale > 0.0f && cmax > rule.max_scale);
  return Cls{!split && !drop, clone && !drop, split && !drop_child};
}

__global__ __launch_bounds__(kDensThreads) void densify_count_kernel(
    int64_t n, const float* __restrict__ scales, const float* __restrict__ opac, const float* __restrict__ grad_sum,
    const float* __restrict__ tau_sum, const int32_t* __restrict__ count, DensRule rule, uint32_t* __restrict__ blockcnt,
    int nblocks) {
  __shared__ uint32_t wcnt[kDensWaves][3];
  const int64_t i = (int64_t)blockIdx.x * kDensThreads + threadIdx.x;
  Cls c{false, false, false};
  if (i < n) c = classify(i, n, scales, opac, grad_sum, tau_sum, count, rule);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t n0 = (uint32_t)__popcll(__ballot(c.orig));
  const uint32_t n1 = (uint32_t)__popcll(__ballot(c.clone));
  const uint32_t n2 = (uint32_t)__popcll(__ballot(c.child));
  if (lane == 0) {
    wcnt[w][0] = n0;
    wcnt[w][1] = n1;
    wcnt[w][2] = n2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kDensWaves; ++k) s += wcnt[k][threadIdx.x];
    blockcnt[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s;
  }
}

// Exclusive scan of the per-block counts of each group (in place); group totals to out_counts
// (originals, clones, first children, second children).
__global__ __launch_bounds__(kScanThreads) void densify_scan_kernel(uint32_t* __restrict__ blockcnt, int nblocks,
                                                                     int64_t* __restrict__ out_counts) {
  __shared__ uint64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int chunk = (nblocks + kScanThreads - 1) / kScanThreads;
  const int b0 = min(nblocks, t * chunk), b1 = min(nblocks, b0 + chunk);
  for (int g = 0; g < 3; ++g) {
    uint32_t* c = blockcnt + (int64_t)g * nblocks;
    uint64_t s = 0;
    for (int b = b0; b < b1; ++b) s += c[b];
    part[t] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the chunk sums
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const uint64_t add = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += add;
      __syncthreads();
    }
    uint64_t run = part[t] - s;
    for (int b = b0; b < b1; ++b) {
      const uint32_t v = c[b];
      c[b] = (uint32_t)run;
      run += v;
    }
    if (t == kScanThreads - 1) {
      out_counts[g] = (int64_t)part[t];
      if (g == 2) out_counts[3] = (int64_t)part[t];
    }
    __syncthreads();
  }
}

template <int K>
__device__ inline void copy_gaussian(int64_t i, int64_t n, int64_t pos, int64_t cap, const float* __restrict__ means,
                                     const float* __restrict__ scales, const float* __restrict__ quats,
                                     const float* __restrict__ opac, const float* __restrict__ sh,
                                     float* __restrict__ om, float* __restrict__ os, float* __restrict__ oq,
                                     float* __restrict__ oo, float* __restrict__ osh, int32_t* __restrict__ osrc) {
#pragma unroll
  for (int k = 0; k < 3; ++k) om[k * cap + pos] = means[k * n + i];
#pragma unroll
  for (int k = 0; k < 3; ++k) os[k * cap + pos] = scales[k * n + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) oq[k * cap + pos] = quats[k * n + i];
  oo[pos] = opac[i];
#pragma unroll
  for (int k = 0; k < K * 3; ++k) osh[k * cap + pos] = sh[k * n + i];
  osrc[pos] = (int32_t)i;
}

template <int K>
__global__ __launch_bounds__(kDensThreads) void densify_scatter_kernel(
    int64_t n, const float* __restrict__ means, const float* __restrict__ scales, const float* __restrict__ quats,
    const float* __restrict__ opac, const float* __restrict__ sh, const float* __restrict__ grad_sum,
    const float* __restrict__ tau_sum, const int32_t* __restrict__ count, const float* __restrict__ noise, DensRule rule,
    const uint32_t* __restrict__ blockoff, int nblocks, const int64_t* __restrict__ totals, int64_t cap,
    float* __restrict__ om, float* __restrict__ os, float* __restrict__ oq, float* __restrict__ oo,
    float* __restrict__ osh, int32_t* __restrict__ osrc) {
  __shared__ uint32_t wcnt[kDensWaves][3];
  const int64_t i = (int64_t)blockIdx.x * kDensThreads + threadIdx.x;
  Cls c{false, false, false};
  if (i < n) c = classify(i, n, scales, opac, grad_sum, tau_sum, count, rule);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t m0 = __ballot(c.orig), m1 = __ballot(c.clone), m2 = __ballot(c.child);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  if (lane == 0) {
    wcnt[w][0] = (uint32_t)__popcll(m0);
    wcnt[w][1] = (uint32_t)__popcll(m1);
    wcnt[w][2] = (uint32_t)__popcll(m2);
  }
  __syncthreads();
  if (i >= n) return;
  uint32_t wo[3] = {0, 0, 0};
  for (int k = 0; k < w; ++k) {
    wo[0] += wcnt[k][0];
    wo[1] += wcnt[k][1];
    wo[2] += wcnt[k][2];
  }
  const int64_t t0 = totals[0], t1 = totals[1], t2 = totals[2];
  if (c.orig) {
    const int64_t pos = (int64_t)blockoff[blockIdx.x] + wo[0] + __popcll(m0 & below);
    copy_gaussian<K>(i, n, pos, cap, means, scales, quats, opac, sh, om, os, oq, oo, osh, osrc);
  }
  if (c.clone) {
    const int64_t pos = t0 + (int64_t)blockoff[nblocks + blockIdx.x] + wo[1] + __popcll(m1 & below);
    copy_gaussian<K>(i, n, pos, cap, means, scales, quats, opac, sh, om, os, oq, oo, osh, osrc);
  }
  if (c.child) {
    const int64_t r = (int64_t)blockoff[2 * (int64_t)nblocks + blockIdx.x] + wo[2] + __popcll(m2 & below);
    // rotation of the normalised quaternion (w, x, y, z)
    float qw = quats[i], qx = quats[n + i], qy = quats[2 * n + i], qz = quats[3 * n + i];
    const float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= inv; qx *= inv; qy *= inv; qz *= inv;
    const float R[9] = {1.0f - 2.0f * (qy * qy + qz * qz), 2.0f * (qx * qy - qw * qz), 2.0f * (qx * qz + qw * qy),
                        2.0f * (qx * qy + qw * qz), 1.0f - 2.0f * (qx * qx + qz * qz), 2.0f * (qy * qz - qw * qx),
                        2.0f * (qx * qz - qw * qy), 2.0f * (qy * qz + qw * qx), 1.0f - 2.0f * (qx * qx + qy * qy)};
    const float s[3] = {scales[i], scales[n + i], scales[2 * n + i]};
    for (int ch = 0; ch < 2; ++ch) {
      const int64_t pos = t0 + t1 + (int64_t)ch * t2 + r;
      copy_gaussian<K>(i, n, pos, cap, means, scales, quats, opac, sh, om, os, oq, oo, osh, osrc);
      const float* xi = noise + (int64_t)ch * 3 * n;
      const float l[3] = {s[0] * xi[i], s[1] * xi[n + i], s[2] * xi[2 * n + i]};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        om[k * cap + pos] = means[k * n + i] + (R[3 * k] * l[0] + R[3 * k + 1] * l[1] + R[3 * k + 2] * l[2]);
        os[k * cap + pos] = s[k] / 1.6f;
      }
    }
  }
}

inline int dens_blocks(int64_t n) { return (int)((n + kDensThreads - 1) / kDensThreads); }

}  // namespace

size_t densify_workspace_bytes(int64_t n) {
  const size_t b = (size_t)3 * (size_t)dens_blocks(n) * sizeof(uint32_t);
  return ((b + 255) / 256) * 256 + 256;
}

hipError_t launch_densify(int64_t n, int32_t sh_degree, const float* means, const float* scales, const float* quats,
                          const float* opac, const float* sh, const float* grad_sum, const float* tau_sum,
                          const int32_t* count, const float* noise, const odgs_densify_params& dp, int64_t capacity,
                          float* out_means, float* out_scales, float* out_quats, float* out_opac, float* out_sh,
                          int32_t* out_src, int64_t* out_counts, void* ws, hipStream_t st) {
  const int nb = dens_blocks(n);
  uint32_t* blockcnt = static_cast<uint32_t*>(ws);
  DensRule rule;
  rule.big = dp.percent_dense * dp.extent;
  rule.min_op = dp.min_opacity;
  rule.max_scale = dp.max_scale_frac > 0.0f ? dp.max_scale_frac * dp.extent : 0.0f;
  if (nb > 0)
    hipLaunchKernelGGL(densify_count_kernel, dim3(nb), dim3(kDensThreads), 0, st, n, scales, opac, grad_sum, tau_sum,
                       count, rule, blockcnt, nb);
  hipLaunchKernelGGL(densify_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, blockcnt, nb, out_counts);
  if (nb > 0) {
#define ODGS_DENS(KK)                                                                                             \
  hipLaunchKernelGGL(densify_scatter_kernel<KK>, dim3(nb), dim3(kDensThreads), 0, st, n, means, scales, quats, opac, \
                     sh, grad_sum, tau_sum, count, noise, rule, blockcnt, nb, out_counts, capacity, out_means,      \
                     out_scales, out_quats, out_opac, out_sh, out_src)
    switch (sh_degree) {
      case 0: ODGS_DENS(1); break;
      case 1: ODGS_DENS(4); break;
      case 2: ODGS_DENS(9); break;
      default: ODGS_DENS(16); break;
    }
#undef ODGS_DENS
  }
  return hipGetLastError();
}

}  // namespace odgs
