// Training step around the rasterizer: the L1 image loss with its gradient, and one Adam update
// of the Gaussian parameters kept before their activations (the 3DGS recipe the paper trains
// with, per its implementation details: scale = exp(raw), opacity = sigmoid(raw), quaternions
// normalised inside the rasterizer).  Both are streaming passes bound by HBM bandwidth.
#include <mutex>

#include "common.h"

namespace odgs {

// Scratch of odgs_l1_loss_noalloc: the per-block partial sums of l1_kernel, kept in a file-scope
// device array so that entry point allocates nothing.  Every GPU the library runs on holds its own
// copy at its own address until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the address hipGetSymbolAddress returns for the current
// device (l1_scratch_ptr), never the array's name.
constexpr int kL1ScratchBlocks = 65536;  // 512 KiB of doubles
static __device__ __align__(256) double scratch[kL1ScratchBlocks];

namespace {

constexpr int kL1Threads = 256;
constexpr int kL1Ipt = 16;
constexpr int kL1Block = kL1Threads * kL1Ipt;

// dL/drgb = sign(rgb - target) / count (sign(0) = 0) and per-block sums of |rgb - target| in
// double (summed in a fixed order by the final kernel, so the loss is reproducible).
__global__ __launch_bounds__(kL1Threads) void l1_kernel(const float* __restrict__ rgb, const float* __restrict__ tgt,
                                                       int64_t count, float inv_count, float* __restrict__ dL,
                                                       double* __restrict__ partial) {
  __shared__ double wsum[kL1Threads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kL1Block;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < kL1Ipt; ++r) {
    const int64_t i = base + r * kL1Threads + threadIdx.x;  // coalesced
    if (i < count) {
      const float d = rgb[i] - tgt[i];
      dL[i] = d > 0.0f ? inv_count : (d < 0.0f ? -inv_count : 0.0f);
      s += (double)fabsf(d);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kL1Threads / kWave; ++w) t += wsum[w];
    partial[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(256) void l1_final_kernel(const double* __restrict__ partial, int nblocks,
                                                       double inv_count, float* __restrict__ loss) {
  __shared__ double wsum[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) s += partial[b];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[0] = (float)(((wsum[0] + wsum[1]) + (wsum[2] + wsum[3])) * inv_count);
}

enum Act { kIdentity = 0, kExp = 1, kSigmoid = 2 };

struct AdamArgs {
  float beta1, beta2, eps;
};

// One Adam update per element (Kingma & Ba, with PyTorch's placement of eps): the gradient with
// respect to the activated value is chained through the activation (using the activated value
// the step's forward pass read), the moments updated, the raw parameter moved, and the activated
// value rewritten for the next forward pass.  The learning rate is lr[g0] for elements below
// `split`, lr[g1] above it (the SH DC planes vs the rest); the step count is read on the device.
template <int ACT>
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ raw, float* __restrict__ act,
                                                   const float* __restrict__ grad, float* __restrict__ m,
                                                   float* __restrict__ v, int64_t count, int64_t split,
                                                   const float* __restrict__ lr, int g0, int g1,
                                                   const int32_t* __restrict__ step, AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float t = (float)(step[0] + 1);
  const float bc1 = 1.0f - powf(a.beta1, t), bc2 = 1.0f - powf(a.beta2, t);
  float g = grad[i];
  if (ACT == kExp) g *= act[i];
  if (ACT == kSigmoid) g *= act[i] * (1.0f - act[i]);
  const float mm = a.beta1 * m[i] + (1.0f - a.beta1) * g;
  const float vv = a.beta2 * v[i] + (1.0f - a.beta2) * (g * g);
  const float rate = lr[i < split ? g0 : g1];
  const float p = raw[i] - (rate / bc1) * mm / (sqrtf(vv) / sqrtf(bc2) + a.eps);
  m[i] = mm;
  v[i] = vv;
  raw[i] = p;
  act[i] = ACT == kExp ? expf(p) : (ACT == kSigmoid ? 1.0f / (1.0f + expf(-p)) : p);
}

__global__ void step_increment_kernel(int32_t* __restrict__ step) {
  if (threadIdx.x == 0) step[0] = step[0] + 1;
}

inline int l1_blocks(int64_t count) { return (int)((count + kL1Block - 1) / kL1Block); }

template <int ACT>
void launch_adam(float* raw, float* act, const float* grad, float* m, float* v, int64_t count, int64_t split,
                 const float* lr, int g0, int g1, const int32_t* step, const AdamArgs& a, hipStream_t st) {
  if (count == 0) return;
  hipLaunchKernelGGL((adam_kernel<ACT>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, raw, act, grad, m,
                     v, count, split, lr, g0, g1, step, a);
}

// Device address of `scratch` on the current device, looked up once per device (with that device
// current) on its first use and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hipError_t l1_scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

int64_t l1_noalloc_max_count() { return (int64_t)kL1ScratchBlocks * kL1Block; }

size_t l1_workspace_bytes(int64_t count) {
  return (((size_t)l1_blocks(count) * sizeof(double) + 255) / 256) * 256 + 256;
}

hipError_t launch_l1(const float* rgb, const float* tgt, int64_t count, float* dL, float* loss, void* ws,
                     hipStream_t st) {
  const int nb = l1_blocks(count);
  double* partial = static_cast<double*>(ws);
  if (nb > 0)
    hipLaunchKernelGGL(l1_kernel, dim3(nb), dim3(kL1Threads), 0, st, rgb, tgt, count,
                       (float)(1.0 / (double)count), dL, partial);
  hipLaunchKernelGGL(l1_final_kernel, dim3(1), dim3(256), 0, st, partial, nb,
                     count > 0 ? 1.0 / (double)count : 0.0, loss);
  return hipGetLastError();
}

hipError_t launch_l1_noalloc(const float* rgb, const float* tgt, int64_t count, float* dL, float* loss,
                             hipStream_t st) {
  if (count > l1_noalloc_max_count()) return hipErrorInvalidValue;
  double* partial = nullptr;
  const hipError_t e = l1_scratch_ptr(&partial);
  if (e != hipSuccess) return e;
  // every block of l1_kernel writes its partial and l1_final_kernel reads exactly those, so the
  // array needs no clearing between calls
  return launch_l1(rgb, tgt, count, dL, loss, partial, st);
}

hipError_t launch_adam_step(int64_t n, int32_t sh_degree, const odgs_param_ptrs& raw, const odgs_param_ptrs& act,
                            const odgs_param_ptrs& grad, const odgs_param_ptrs& m, const odgs_param_ptrs& v,
                            const float* lr, int32_t* step, const odgs_adam_hyper& hp, hipStream_t st) {
  const AdamArgs a{hp.beta1, hp.beta2, hp.eps};
  const int64_t K = (int64_t)(sh_degree + 1) * (sh_degree + 1);
  launch_adam<kIdentity>(raw.means, act.means, grad.means, m.means, v.means, 3 * n, 3 * n, lr, 0, 0, step, a, st);
  launch_adam<kExp>(raw.scales, act.scales, grad.scales, m.scales, v.scales, 3 * n, 3 * n, lr, 1, 1, step, a, st);
  launch_adam<kIdentity>(raw.quats, act.quats, grad.quats, m.quats, v.quats, 4 * n, 4 * n, lr, 2, 2, step, a, st);
  launch_adam<kSigmoid>(raw.opacities, act.opacities, grad.opacities, m.opacities, v.opacities, n, n, lr, 3, 3, step,
                        a, st);
  launch_adam<kIdentity>(raw.sh, act.sh, grad.sh, m.sh, v.sh, 3 * K * n, 3 * n, lr, 4, 5, step, a, st);
  hipLaunchKernelGGL(step_increment_kernel, dim3(1), dim3(64), 0, st, step);
  return hipGetLastError();
}

}  // namespace odgs
