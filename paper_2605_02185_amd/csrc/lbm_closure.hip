// gfx950 kernels of the learned boundary closure: a 36 -> 64 -> 64 -> 3
// GELU MLP on the matrix cores (bfloat16 operands, FP32 accumulation), its
// training step (forward, backward, fixed-order gradient reduction, Adam),
// the sampler that cuts training data out of a full-domain run, and the
// per-step closure that predicts the missing populations on the open
// boundaries of a truncated domain.
//
// Boundary nodes of a lattice (nx x ny) are numbered
//   [0, nx-2)                  top row    y = ny-1, x = 1 + i
//   [nx-2, 2(nx-2))            bottom row y = 0,    x = 1 + i - (nx-2)
//   [2(nx-2), 2(nx-2) + ny-2)  outlet     x = nx-1, y = 1 + i - 2(nx-2)
// Each boundary is seen in a canonical frame whose outward normal is +y (the
// bottom mirrored, the outlet rotated by a quarter turn), where the missing
// populations are always S, SW and SE; one network serves all three.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <mutex>

#include "lbm_internal.h"

namespace lbm {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MB = 32;  // samples per block

// Round to the nearest bfloat16, ties to even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// SplitMix64 (Steele, Lea & Flood 2014) as a counter-based generator, and a
// standard normal variate from one 64-bit draw by the Box-Muller transform.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ float gauss(uint64_t key) {
  const uint64_t r = splitmix64(key);
  const float u1 = (float)((r >> 40) + 1) * (1.0f / 16777217.0f);  // (0, 1]
  const float u2 = (float)((r >> 16) & 0xFFFFFFull) * (1.0f / 16777216.0f);
  return sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// C (16 x 16, FP32) += A (16 x K) B (K x 16), bfloat16 operands, K a multiple
// of 16.  A(i, k) = pa[i*sai + k*sak], B(k, n) = pb[k*sbk + n*sbn].  Lane l
// supplies A row l%16 and B column l%16 at k = k0 + 4(l/16) .. +3, and holds
// C rows 4(l/16) .. +3 of column l%16.
__device__ __forceinline__ f32x4 tile_mma(const uint16_t* pa, int sai, int sak, const uint16_t* pb,
                                          int sbk, int sbn, int K, f32x4 c) {
  const int l = threadIdx.x & 63;
  const int i = l & 15, kq = (l >> 4) * 4;
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = (short)pa[i * sai + (k0 + kq + j) * sak];
      b[j] = (short)pb[(k0 + kq + j) * sbk + i * sbn];
    }
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
  }
  return c;
}

__device__ __forceinline__ int out_row(int j) { return 4 * ((threadIdx.x & 63) >> 4) + j; }
__device__ __forceinline__ int out_col() { return threadIdx.x & 15; }

struct MlpLds {
  uint16_t x[MB * 48];   // inputs, K padded to 48
  uint16_t h1[MB * 64];
  uint16_t h2[MB * 64];
  uint16_t dz[MB * 64];
  uint16_t dy[MB * 16];
  float g1[MB * 64];     // gelu'(z1), later dz1
  float g2[MB * 64];     // gelu'(z2), later dz2
  float y[MB * 16];      // outputs, later dy
};

// Forward pass of the MB samples staged in s.x.  Weights: W1b [48][64],
// W2b [64][64], W3b [64][16] (bfloat16, row-major input x output, zero
// padded); biases FP32.  Keeps gelu' for the backward pass when `train`.
__device__ __forceinline__ void forward_block(MlpLds& s, const uint16_t* W1b, const uint16_t* W2b,
                                              const uint16_t* W3b, const float* b1, const float* b2,
                                              const float* b3, bool train) {
  const int w = threadIdx.x >> 6;
  for (int t = w; t < 8; t += 4) {  // layer 1: 2 x 4 tiles
    const int rb = t >> 2, cb = t & 3;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.x + rb * 16 * 48, 48, 1, W1b + cb * 16, 64, 1, 48, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rb * 16 + out_row(j), n = cb * 16 + out_col();
      const float z = c[j] + b1[n];
      s.h1[r * 64 + n] = to_bf16(gelu(z));
      if (train) s.g1[r * 64 + n] = gelu_grad(z);
    }
  }
  __syncthreads();
  for (int t = w; t < 8; t += 4) {  // layer 2
    const int rb = t >> 2, cb = t & 3;
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.h1 + rb * 16 * 64, 64, 1, W2b + cb * 16, 64, 1, 64, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = rb * 16 + out_row(j), n = cb * 16 + out_col();
      const float z = c[j] + b2[n];
      s.h2[r * 64 + n] = to_bf16(gelu(z));
      if (train) s.g2[r * 64 + n] = gelu_grad(z);
    }
  }
  __syncthreads();
  if (w < 2) {  // layer 3: 2 tiles, 3 of 16 columns used
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = tile_mma(s.h2 + w * 16 * 64, 64, 1, W3b, 16, 1, 64, c);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = w * 16 + out_row(j), n = out_col();
      s.y[r * 16 + n] = n < 3 ? c[j] + b3[n] : 0.0f;
    }
  }
  __syncthreads();
}

constexpr int kWb = 48 * 64 + 64 * 64 + 64 * 16;  // bfloat16 weights, padded layouts

// Copies the bfloat16 weights into LDS with 16-byte loads (8192 halves).
__device__ __forceinline__ void stage_weights(uint16_t* dst, const uint16_t* __restrict__ Wb) {
  const uint4* src = (const uint4*)Wb;
  uint4* d = (uint4*)dst;
  for (int i = threadIdx.x; i < kWb / 8; i += blockDim.x) d[i] = src[i];
}

// Offsets of the parameters in the flat FP32 vector (W row-major in x out).
constexpr int OW1 = 0, OB1 = 2304, OW2 = 2368, OB2 = 6464, OW3 = 6528, OB3 = 6720, NP = 6723;

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
  forward_block(s, W1b, W2b, W3b, master + OB1, master + OB2, master + OB3, true);
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
  forward_block(s, wl, wl + 48 * 64, wl + 48 * 64 + 64 * 64, master + OB1, master + OB2, master + OB3, false);
  for (int e = tid; e < MB * 3; e += 256) {
    const int r = e / 3, c = e % 3, smp = blk * MB + r;
    if (smp < M) Y[(int64_t)smp * 3 + c] = norm ? s.y[r * 16 + c] * norm[72 + c] : s.y[r * 16 + c];
  }
}

// ----------------------------------------------------------- boundary data
// Physical direction of canonical direction c for each boundary type
// (0 top: identity; 1 bottom: mirror in y; 2 outlet: quarter turn).
__constant__ int kCanon[3][9] = {{0, 1, 2, 3, 4, 5, 6, 7, 8},
                                 {0, 1, 4, 3, 2, 8, 7, 6, 5},
                                 {0, 4, 1, 2, 3, 8, 5, 6, 7}};

struct BNode {
  int type, x, y, nx_, ny_;  // boundary type, node, inward step (nx_, ny_)
};

__device__ __forceinline__ BNode boundary_node(int i, int nx, int ny) {
  BNode b;
  if (i < nx - 2) {
    b = {0, 1 + i, ny - 1, 0, -1};
  } else if (i < 2 * (nx - 2)) {
    b = {1, 1 + i - (nx - 2), 0, 0, 1};
  } else {
    b = {2, nx - 1, 1 + i - 2 * (nx - 2), -1, 0};
  }
  return b;
}

__device__ __forceinline__ float ld(const float* __restrict__ A, const Geometry& g, int k, int x, int y) {
  return A[(int64_t)k * g.plane + (int64_t)y * g.pitch + x];
}

// The 36 features of a boundary node: for the node and its two inward
// neighbours, the nine stored post-collision deviations f*_k - w_k in
// canonical order, then drho = rho - 1 and the canonical velocity.  (ox, oy)
// places the boundary node's lattice inside the state's lattice.
__device__ __forceinline__ void layer_features(const float* __restrict__ A, const Geometry& g, const BNode& b,
                                               int ox, int oy, int L, float* f) {
  const int x = ox + b.x + L * b.nx_, y = oy + b.y + L * b.ny_;
  float h[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) h[k] = ld(A, g, k, x, y);
  const float drho = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
  const float ir = 1.0f / (1.0f + drho);
  const float u = (((h[1] - h[3]) + (h[5] - h[7])) + (h[8] - h[6])) * ir;
  const float v = (((h[2] - h[4]) + (h[5] - h[7])) + (h[6] - h[8])) * ir;
#pragma unroll
  for (int c = 0; c < 9; ++c) f[c] = h[kCanon[b.type][c]];
  f[9] = drho;
  f[10] = b.type == 2 ? -v : u;
  f[11] = b.type == 0 ? v : (b.type == 1 ? -v : u);
}

__device__ void features(const float* __restrict__ A, const Geometry& g, const BNode& b, int ox, int oy,
                         float* f) {
  for (int L = 0; L < 3; ++L) layer_features(A, g, b, ox, oy, L, f + 12 * L);
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

// The closure of one step: features of MB boundary nodes of the state A,
// z-scored, through the network; residual r = y * scale (physical order of
// the missing populations of each boundary).
// Boundaries whose bit is clear in `mask` (1 top, 2 bottom, 4 outlet) keep
// the plain treatment: their residuals are written as zero.  With beta < 1
// the applied residual follows the prediction through a first-order
// low-pass, r <- r + beta (prediction - r), per node.  With limit > 0 the
// network's output is clamped to [-limit, limit] before it is scaled (so the
// residual stays within limit times the training targets' spread), and
// outlet nodes within outlet_taper nodes of the top and bottom rows keep
// the plain treatment.
__global__ __launch_bounds__(256) void closure_kernel(const float* __restrict__ A, Geometry g, int nb,
                                                      const uint16_t* __restrict__ Wb,
                                                      const float* __restrict__ master,
                                                      const float* __restrict__ norm, int mask, float beta,
                                                      int taper, float limit, int outlet_taper,
                                                      int outlet_neutral, const float* __restrict__ bias,
                                                      float* __restrict__ resid) {
  __shared__ MlpLds s;
  __shared__ __align__(16) uint16_t wl[kWb];
  const int blk = blockIdx.x, tid = threadIdx.x;
  stage_weights(wl, Wb);
  if (tid < MB * 3) {  // thread (node r, layer L): 12 features
    const int r = tid / 3, L = tid % 3, i = blk * MB + r;
    float f[12];
    if (i < nb) {
      const BNode b = boundary_node(i, g.nx, g.ny);
      layer_features(A, g, b, 0, 0, L, f);
    }
    for (int c = 0; c < 12; ++c) {
      const int q = L * 12 + c;
      const float v = i < nb ? (f[c] - norm[q]) * norm[36 + q] : 0.0f;
      s.x[r * 48 + q] = to_bf16(v);
    }
  } else if (tid < MB * 3 + MB) {  // zero the K padding 36..47
    const int r = tid - MB * 3;
    for (int c = 36; c < 48; ++c) s.x[r * 48 + c] = 0;
  }
  __syncthreads();
  forward_block(s, wl, wl + 48 * 64, wl + 48 * 64 + 64 * 64, master + OB1, master + OB2, master + OB3, false);
  if (tid < MB * 3) {
    const int r = tid / 3, c = tid % 3, i = blk * MB + r;
    if (i < nb) {
      const BNode b = boundary_node(i, g.nx, g.ny);
      // rows keep the plain treatment within `taper` nodes of the inlet and outlet
      const bool on = ((mask >> b.type) & 1) &&
                      (b.type == 2 ? (b.y >= outlet_taper && b.y <= g.ny - 1 - outlet_taper)
                                   : (b.x >= taper && b.x <= g.nx - 1 - taper));
      // one output: the clamped network value times its scale, plus the
      // node's fixed part when a per-node bias is set
      auto out = [&](int j) {
        float y = s.y[r * 16 + j];
        if (limit > 0.0f) y = fminf(fmaxf(y, -limit), limit);
        return bias ? y * norm[72 + j] + bias[(int64_t)i * 3 + j] : y * norm[72 + j];
      };
      float pred = on ? out(c) : 0.0f;
      if (on && outlet_neutral && b.type == 2) {
        // remove the part that changes the node's mass: the three residuals
        // then sum to zero (and so does the x-momentum they carry)
        pred -= (out(0) + out(1) + out(2)) * (1.0f / 3.0f);
      }
      float* dst = resid + (int64_t)i * 3 + c;
      *dst = beta >= 1.0f ? pred : *dst + beta * (pred - *dst);
    }
  }
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

hipError_t launch_closure(const float* A, const Geometry& g, const uint16_t* Wb, const float* master,
                          const float* norm, int mask, float beta, int taper, float limit, int outlet_taper,
                          int outlet_neutral, const float* bias, float* resid, hipStream_t s) {
  const int nb = 2 * (g.nx - 2) + (g.ny - 2);
  hipLaunchKernelGGL(closure_kernel, dim3((nb + MB - 1) / MB), dim3(256), 0, s, A, g, nb, Wb, master, norm,
                     mask, beta, taper, limit, outlet_taper, outlet_neutral, bias, resid);
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
