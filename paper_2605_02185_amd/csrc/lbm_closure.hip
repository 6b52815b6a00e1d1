// gfx950 kernels of the learned boundary closure: a 36 -> 64 -> 64 -> 3
// GELU MLP on the matrix cores (bfloat16 operands, FP32 accumulation), its
// training step (forward, backward, fixed-order gradient reduction, Adam),
// the sampler that cuts training data out of a full-domain run, and the
// per-step closure that predicts the missing populations on the open
// boundaries of a truncated domain.
//
// The network's forward pass, the boundary numbering and features and the
// closure block are in lbm_mlp_dev.h (shared with the step kernel that runs
// the closure in its own launch).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "lbm_internal.h"
#include "lbm_mlp_dev.h"

namespace lbm {
namespace {


// One block: MB samples (rows idx[blk*MB + r] of X and T, or row blk*MB + r
// when idx is null; rows beyond B are padding).  Writes the block's gradient
// (FP32, flat layout) and its sum of squared errors.
// With `norm` (feature mean[36], 1/std[36], output scale[3]) the raw X and
// T are z-scored on load: x = (X - mean)/std, t = T/scale.  With noise > 0
// every (z-scored) input gets independent N(0, noise^2) noise keyed by
// (key, dataset row, feature), which regularises the fit towards maps that
// do not amplify small input errors.
__global__ __launch_bounds__(256) void mlp_train_kernel(const float* __restrict__ X, const float* __restrict__ T,
                                                        const int* __restrict__ idx, int B,
                                                        const uint16_t* __restrict__ Wb,
                                                        const float* __restrict__ master,
                                                        const float* __restrict__ norm,
                                                        float* __restrict__ gpart, double* __restrict__ lpart,
                                                        float dscale, float noise, uint64_t key) {
  __shared__ MlpLds s;
  __shared__ double red[256];
  __shared__ __align__(16) uint16_t wl[kWb];
  const int blk = blockIdx.x, tid = threadIdx.x, w = tid >> 6;
  stage_weights(wl, Wb);
  const uint16_t *W1b = wl, *W2b = wl + 48 * 64, *W3b = W2b + 64 * 64;
  for (int e = tid; e < MB * 48; e += 256) {
    const int r = e / 48, c = e % 48, smp = blk * MB + r;
    float v = 0.0f;
    if (smp < B && c < 36) {
      const int64_t row = idx ? idx[smp] : smp;
      v = X[row * 36 + c];
      if (norm) v = (v - norm[c]) * norm[36 + c];
      if (noise > 0.0f) v += noise * gauss(key ^ (uint64_t)(row * 64 + c));
    }
    s.x[e] = to_bf16(v);
  }
  __syncthreads();
  forward_block<true>(s, W1b, W2b, W3b, master + OB1, master + OB2, master + OB3);
  // dy = 2 (y - t)/(3 B) in FP32 (kept in s.y) and in bfloat16 (s.dy)
  double sq = 0.0;
  for (int e = tid; e < MB * 16; e += 256) {
    const int r = e / 16, c = e % 16, smp = blk * MB + r;
    float d = 0.0f;
    if (smp < B && c < 3) {
      float tv = T[(int64_t)(idx ? idx[smp] : smp) * 3 + c];
      if (norm) tv = tv / norm[72 + c];
      const float diff = s.y[e] - tv;
      sq += (double)diff * diff;
      d = dscale * diff;
    }
    s.y[e] = d;
    s.dy[e] = to_bf16(d);
  }
  red[tid] = sq;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) lpart[blk] = red[0];
  float* g = gpart + (int64_t)blk * NP;
  {  // dW3 = h2^T dy: 4 tiles of [64 in x 16 out], K = MB samples
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.h2 + w * 16, 1, 64, s.dy, 16, 1, MB, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = w * 16 + out_row(j), n = out_col();
      if (n < 3) g[OW3 + i * 3 + n] = c[j];
    }
  }
  if (tid < 3) {
    float sum = 0.0f;
    for (int r = 0; r < MB; ++r) sum += s.y[r * 16 + tid];
    g[OB3 + tid] = sum;
  }
  for (int t = w; t < 8; t += 4) {  // dh2 = dy W3^T, dz2 = dh2 gelu'(z2)
    const int rb = t >> 2, cb = t & 3;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.dy + rb * 16 * 16, 16, 1, W3b + cb * 16 * 16, 1, 16, 16, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rb * 16 + out_row(j), n = cb * 16 + out_col();
      const float dz = c[j] * s.g2[r * 64 + n];
      s.g2[r * 64 + n] = dz;
      s.dz[r * 64 + n] = to_bf16(dz);
    }
  }
  __syncthreads();
  for (int t = w; t < 16; t += 4) {  // dW2 = h1^T dz2
    const int ib = t >> 2, cb = t & 3;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.h1 + ib * 16, 1, 64, s.dz + cb * 16, 64, 1, MB, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) g[OW2 + (ib * 16 + out_row(j)) * 64 + cb * 16 + out_col()] = c[j];
  }
  if (tid < 64) {
    float sum = 0.0f;
    for (int r = 0; r < MB; ++r) sum += s.g2[r * 64 + tid];
    g[OB2 + tid] = sum;
  }
  for (int t = w; t < 8; t += 4) {  // dh1 = dz2 W2^T, dz1 = dh1 gelu'(z1) (into h2 / g1)
    const int rb = t >> 2, cb = t & 3;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.dz + rb * 16 * 64, 64, 1, W2b + cb * 16 * 64, 1, 64, 64, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rb * 16 + out_row(j), n = cb * 16 + out_col();
      const float dz = c[j] * s.g1[r * 64 + n];
      s.g1[r * 64 + n] = dz;
      s.h2[r * 64 + n] = to_bf16(dz);
    }
  }
  __syncthreads();
  for (int t = w; t < 12; t += 4) {  // dW1 = x^T dz1: 3 x 4 tiles, rows 36..47 dropped
    const int ib = t >> 2, cb = t & 3;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.x + ib * 16, 1, 48, s.h2 + cb * 16, 64, 1, MB, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int i = ib * 16 + out_row(j);
      if (i < 36) g[OW1 + i * 64 + cb * 16 + out_col()] = c[j];
    }
  }
  if (tid < 64) {
    float sum = 0.0f;
    for (int r = 0; r < MB; ++r) sum += s.g1[r * 64 + tid];
    g[OB1 + tid] = sum;
  }
}

// Sums the block gradients in block order (FP64), optionally applies one
// Adam step (step >= 1) to the FP32 master weights, and refreshes the
// bfloat16 copies.  With step == 0 it only reduces (into grad_out).
__global__ __launch_bounds__(256) void mlp_adam_kernel(const float* __restrict__ gpart, int nblk,
                                                       const double* __restrict__ lpart, float* master,
                                                       float* m, float* v, uint16_t* Wb, float* grad_out,
                                                       double* loss_out, int step, float lr, float b1,
                                                       float b2, float eps, double inv_count) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p == 0 && loss_out) {
    double l = 0.0;
    for (int b = 0; b < nblk; ++b) l += lpart[b];
    *loss_out = l * inv_count;
  }
  if (p >= NP) return;
  double gs = 0.0;
  for (int b = 0; b < nblk; ++b) gs += (double)gpart[(int64_t)b * NP + p];
  const float gr = (float)gs;
  if (grad_out) grad_out[p] = gr;
  if (step > 0) {
    const float mm = b1 * m[p] + (1.0f - b1) * gr;
    const float vv = b2 * v[p] + (1.0f - b2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (float)(1.0 - pow((double)b1, (double)step));
    const float vh = vv / (float)(1.0 - pow((double)b2, (double)step));
    master[p] -= lr * mh / (sqrtf(vh) + eps);
  }
  const float wv = master[p];
  if (p < OB1) {
    Wb[(p / 64) * 64 + p % 64] = to_bf16(wv);
  } else if (p >= OW2 && p < OB2) {
    Wb[48 * 64 + (p - OW2)] = to_bf16(wv);
  } else if (p >= OW3 && p < OB3) {
    const int q = p - OW3;
    Wb[48 * 64 + 64 * 64 + (q / 3) * 16 + q % 3] = to_bf16(wv);
  }
}

// With `norm` the inputs are z-scored and the outputs scaled back (y * scale).
__global__ __launch_bounds__(256) void mlp_forward_kernel(const float* __restrict__ X, int M,
                                                          const uint16_t* __restrict__ Wb,
                                                          const float* __restrict__ master,
                                                          const float* __restrict__ norm,
                                                          float* __restrict__ Y) {
  __shared__ MlpLds s;
  __shared__ __align__(16) uint16_t wl[kWb];
  const int blk = blockIdx.x, tid = threadIdx.x;
  stage_weights(wl, Wb);
  for (int e = tid; e < MB * 48; e += 256) {
    const int r = e / 48, c = e % 48, smp = blk * MB + r;
    float v = 0.0f;
    if (smp < M && c < 36) {
      v = X[(int64_t)smp * 36 + c];
      if (norm) v = (v - norm[c]) * norm[36 + c];
    }
    s.x[e] = to_bf16(v);
  }
  __syncthreads();
  forward_block<false>(s, wl, wl + 48 * 64, wl + 48 * 64 + 64 * 64, master + OB1, master + OB2, master + OB3);
  for (int e = tid; e < MB * 3; e += 256) {
    const int r = e / 3, c = e % 3, smp = blk * MB + r;
    if (smp < M) Y[(int64_t)smp * 3 + c] = norm ? s.y[r * 16 + c] * norm[72 + c] : s.y[r * 16 + c];
  }
}

// Training samples from a full-domain state A: for window boundary node
// nodes[s] of a wnx x wny window at offset (ox, oy), the features and the
// residual (population that actually streams in minus the value the plain
// treatment gives) of the canonical S, SW, SE populations.  The plain
// treatments: free-slip for the top and bottom rows (Eq. 7), extrapolation of
// the missing populations from the column inside for the outlet (Eq. 13).
__global__ void sample_kernel(const float* __restrict__ A, Geometry g, int ox, int oy, int wnx, int wny,
                              const int* __restrict__ nodes, int n, const float* __restrict__ bias,
                              float* __restrict__ feat, float* __restrict__ target) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int node = nodes[s];
  if (node < 0 || node >= 2 * (wnx - 2) + (wny - 2)) {  // invalid index: zero sample
    for (int c = 0; c < 36; ++c) feat[(int64_t)s * 36 + c] = 0.0f;
    for (int j = 0; j < 3; ++j) target[(int64_t)s * 3 + j] = 0.0f;
    return;
  }
  const BNode b = boundary_node(node, wnx, wny);
  float f[36];
  features(A, g, b, ox, oy, f);
  for (int c = 0; c < 36; ++c) feat[(int64_t)s * 36 + c] = f[c];
  const int X = ox + b.x, Y = oy + b.y;
  // canonical S, SW, SE and their physical directions
  const int cs[3] = {4, 7, 8};
  for (int j = 0; j < 3; ++j) {
    const int k = kCanon[b.type][cs[j]];
    // true: streamed in from outside the window, f*_k(x - c_k)
    const int cxk = (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0);
    const int cyk = (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0);
    const float truth = ld(A, g, k, X - cxk, Y - cyk);
    float plain;
    if (b.type == 2) {
      // outlet: the value k streams into the node one column inside
      plain = ld(A, g, k, X - 1 - cxk, Y - cyk);
    } else {
      // free-slip: the mirror image in y of k arrives from inside
      const int km = k == 4 ? 2 : k == 7 ? 6 : k == 8 ? 5 : k == 2 ? 4 : k == 6 ? 7 : 8;
      const int cxm = (km == 1 || km == 5 || km == 8) ? 1 : ((km == 3 || km == 6 || km == 7) ? -1 : 0);
      const int cym = (km == 2 || km == 5 || km == 6) ? 1 : ((km == 4 || km == 7 || km == 8) ? -1 : 0);
      plain = ld(A, g, km, X - cxm, Y - cym);
    }
    target[(int64_t)s * 3 + j] = truth - plain - (bias ? bias[(int64_t)node * 3 + j] : 0.0f);
  }
}

// The closure as a kernel of its own (closure_block per block).
__global__ __launch_bounds__(256) void closure_kernel(const float* __restrict__ A, Geometry g, ClosureEval e) {
  __shared__ FwdLds s;
  __shared__ __align__(16) uint16_t wl[kWb];
  closure_block(e, A, g, (int)blockIdx.x, s, wl);
}

// Column sums (out[c]) and sums of squares (out[ncols + c]), FP64, of
// X [M][ncols]; one block per column, each writing only its own two entries.
__global__ __launch_bounds__(256) void column_moments_kernel(const float* __restrict__ X, int64_t M,
                                                             int ncols, double* out) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < M; i += 256) {
    const double v = X[i * ncols + c];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] += s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[c] = s1[0];
    out[ncols + c] = s2[0];
  }
}

}  // namespace

int mlp_blocks(int64_t B) { return (int)((B + MB - 1) / MB); }

hipError_t launch_mlp_train(const float* X, const float* T, const int* idx, int B, const uint16_t* Wb,
                            const float* master, const float* norm, float* gpart, double* lpart, float noise,
                            uint64_t key, hipStream_t s) {
  const float dscale = 2.0f / (3.0f * (float)B);
  hipLaunchKernelGGL(mlp_train_kernel, dim3(mlp_blocks(B)), dim3(256), 0, s, X, T, idx, B, Wb, master, norm,
                     gpart, lpart, dscale, noise, key);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const float* gpart, int nblk, const double* lpart, float* master, float* m, float* v,
                           uint16_t* Wb, float* grad_out, double* loss_out, int step, float lr,
                           double inv_count, hipStream_t s) {
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, s, gpart, nblk, lpart, master, m,
                     v, Wb, grad_out, loss_out, step, lr, 0.9f, 0.999f, 1e-8f, inv_count);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* X, int M, const uint16_t* Wb, const float* master, const float* norm,
                              float* Y, hipStream_t s) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3(mlp_blocks(M)), dim3(256), 0, s, X, M, Wb, master, norm, Y);
  return hipGetLastError();
}

hipError_t launch_sample_boundary(const float* A, const Geometry& g, int ox, int oy, int wnx, int wny,
                                  const int* nodes, int n, const float* bias, float* feat, float* target,
                                  hipStream_t s) {
  hipLaunchKernelGGL(sample_kernel, dim3((n + 63) / 64), dim3(64), 0, s, A, g, ox, oy, wnx, wny, nodes, n,
                     bias, feat, target);
  return hipGetLastError();
}

int closure_blocks(int nb) { return (nb + MB - 1) / MB; }

size_t closure_lds_bytes() { return sizeof(FwdLds) + sizeof(uint16_t) * kWb; }

hipError_t launch_closure(const float* A, const Geometry& g, const ClosureEval& e, hipStream_t s) {
  hipLaunchKernelGGL(closure_kernel, dim3((unsigned)closure_blocks(e.nb)), dim3(256), 0, s, A, g, e);
  return hipGetLastError();
}

hipError_t launch_column_moments(const float* X, int64_t M, int ncols, double* out, hipStream_t s) {
  hipLaunchKernelGGL(column_moments_kernel, dim3(ncols), dim3(256), 0, s, X, M, ncols, out);
  return hipGetLastError();
}

}  // namespace lbm

// ------------------------------------------------ allocation-free moments
// The partial results of lbm_column_moments_noalloc live in this array
// instead of a per-call device allocation.  Host code never uses its name as
// an address: each device's copy is looked up once with hipGetSymbolAddress
// and that pointer is what kernels and copies receive.
namespace {

constexpr int kScratchCols = 4096;
static __device__ __align__(256) double scratch[2 * kScratchCols];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (looked up on first use), or an error.
lbm_status scratch_on_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return lbm::set_error(LBM_ERR_INVALID_ARG, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char m[160];
      snprintf(m, sizeof m, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
      return lbm::set_error(LBM_ERR_HIP, m);
    }
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

}  // namespace

extern "C" lbm_status lbm_column_moments_noalloc(const float* x, int64_t M, int32_t ncols, double* mean,
                                                 double* std, void* stream) {
  if (!x || M < 1 || !mean || !std) return lbm::set_error(LBM_ERR_INVALID_ARG, "bad moments arguments");
  if (ncols < 1 || ncols > kScratchCols) {
    char m[128];
    snprintf(m, sizeof m, "ncols %d outside [1, %d], the columns the static scratch holds", (int)ncols,
             kScratchCols);
    return lbm::set_error(LBM_ERR_INVALID_ARG, m);
  }
  double* d = nullptr;
  lbm_status st = scratch_on_current_device(&d);
  if (st != LBM_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // every entry the kernel's blocks write is its own: nothing to clear first
  hipError_t e = lbm::launch_column_moments(x, M, ncols, d, s);
  if (e == hipSuccess) e = hipMemcpyAsync(mean, d, sizeof(double) * ncols, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(std, d + ncols, sizeof(double) * ncols, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return lbm::set_error(LBM_ERR_HIP, hipGetErrorString(e));
  // the sums sit in mean[] and std[]: turn them into the moments in place
  for (int c = 0; c < ncols; ++c) {
    const double a = mean[c] / (double)M, b = std[c] / (double)M;
    mean[c] = a;
    std[c] = std::sqrt(std::max(0.0, b - a * a));
  }
  return LBM_OK;
}
