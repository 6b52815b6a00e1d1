// Device code shared by the closure kernels (lbm_closure.hip) and the step
// kernel that evaluates the network in the same launch as the steps
// (lbm_kernels.hip): the 36 -> 64 -> 64 -> 3 GELU network on the matrix
// cores (bfloat16 operands, FP32 accumulation), the boundary features and
// one block of the closure evaluation.  Boundary nodes of a lattice
// (nx x ny) are numbered
//   [0, nx-2)                  top row    y = ny-1, x = 1 + i
//   [nx-2, 2(nx-2))            bottom row y = 0,    x = 1 + i - (nx-2)
//   [2(nx-2), 2(nx-2) + ny-2)  outlet     x = nx-1, y = 1 + i - 2(nx-2)
// Each boundary is seen in a canonical frame whose outward normal is +y (the
// bottom mirrored, the outlet rotated by a quarter turn), where the missing
// populations are always S, SW and SE; one network serves all three.
#pragma once

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
// padded); biases FP32.  Keeps gelu' for the backward pass when TRAIN (L is
// MlpLds then; FwdLds, without those arrays, serves inference).
template <bool TRAIN, class L>
__device__ __forceinline__ void forward_block(L& s, const uint16_t* W1b, const uint16_t* W2b,
                                              const uint16_t* W3b, const float* b1, const float* b2,
                                              const float* b3) {
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
      if constexpr (TRAIN) s.g1[r * 64 + n] = gelu_grad(z);
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
      if constexpr (TRAIN) s.g2[r * 64 + n] = gelu_grad(z);
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

// What inference alone needs in LDS (13 KB against MlpLds's 35 KB).
struct FwdLds {
  uint16_t x[MB * 48];
  uint16_t h1[MB * 64];
  uint16_t h2[MB * 64];
  float y[MB * 16];
};

constexpr int kWb = 48 * 64 + 64 * 64 + 64 * 16;  // bfloat16 weights, padded layouts

// Copies the bfloat16 weights into LDS with 16-byte loads (8192 halves).
__device__ __forceinline__ void stage_weights(uint16_t* dst, const uint16_t* __restrict__ Wb) {
  const uint4* src = (const uint4*)Wb;
  uint4* d = (uint4*)dst;
  for (int i = threadIdx.x; i < kWb / 8; i += blockDim.x) d[i] = src[i];
}

// Offsets of the parameters in the flat FP32 vector (W row-major in x out).
constexpr int OW1 = 0, OB1 = 2304, OW2 = 2368, OB2 = 6464, OW3 = 6528, OB3 = 6720, NP = 6723;

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


// One block (256 threads) of the closure: MB boundary nodes from blk * MB on,
// features of the state A, z-scored, through the network; residual r =
// y * scale (physical order of the missing populations of each boundary).
// Boundaries whose bit is clear in `mask` (1 top, 2 bottom, 4 outlet) keep
// the plain treatment: their residuals are written as zero.  With beta < 1
// the applied residual follows the prediction through a first-order
// low-pass per node, resid = resid_in + beta (prediction - resid_in), where
// resid_in holds the residuals in use (it may be resid itself; with beta = 1
// it is not read).  With limit > 0 the network's output is clamped to
// [-limit, limit] before it is scaled (so the residual stays within limit
// times the training targets' spread), and outlet nodes within outlet_taper
// nodes of the top and bottom rows keep the plain treatment.  Every thread
// of the block must call it (it synchronises the block).
__device__ __forceinline__ void closure_block(const ClosureEval& e, const float* __restrict__ A, const Geometry& g,
                                              int blk, FwdLds& s, uint16_t* wl) {
  const int tid = threadIdx.x, nb = e.nb;
  stage_weights(wl, e.Wb);
  if (tid < MB * 3) {  // thread (node r, layer L): 12 features
    const int r = tid / 3, L = tid % 3, i = blk * MB + r;
    float f[12];
    if (i < nb) {
      const BNode b = boundary_node(i, g.nx, g.ny);
      layer_features(A, g, b, 0, 0, L, f);
    }
    for (int c = 0; c < 12; ++c) {
      const int q = L * 12 + c;
      const float v = i < nb ? (f[c] - e.norm[q]) * e.norm[36 + q] : 0.0f;
      s.x[r * 48 + q] = to_bf16(v);
    }
  } else if (tid < MB * 3 + MB) {  // zero the K padding 36..47
    const int r = tid - MB * 3;
    for (int c = 36; c < 48; ++c) s.x[r * 48 + c] = 0;
  }
  __syncthreads();
  forward_block<false>(s, wl, wl + 48 * 64, wl + 48 * 64 + 64 * 64, e.master + OB1, e.master + OB2,
                       e.master + OB3);
  if (tid < MB * 3) {
    const int r = tid / 3, c = tid % 3, i = blk * MB + r;
    if (i < nb) {
      const BNode b = boundary_node(i, g.nx, g.ny);
      // rows keep the plain treatment within `taper` nodes of the inlet and outlet
      const bool on = ((e.mask >> b.type) & 1) &&
                      (b.type == 2 ? (b.y >= e.outlet_taper && b.y <= g.ny - 1 - e.outlet_taper)
                                   : (b.x >= e.taper && b.x <= g.nx - 1 - e.taper));
      // one output: the clamped network value times its scale, plus the
      // node's fixed part when a per-node bias is set
      auto out = [&](int j) {
        float y = s.y[r * 16 + j];
        if (e.limit > 0.0f) y = fminf(fmaxf(y, -e.limit), e.limit);
        return e.bias ? y * e.norm[72 + j] + e.bias[(int64_t)i * 3 + j] : y * e.norm[72 + j];
      };
      float pred = on ? out(c) : 0.0f;
      if (on && e.outlet_neutral && b.type == 2) {
        // remove the part that changes the node's mass: the three residuals
        // then sum to zero (and so does the x-momentum they carry)
        pred -= (out(0) + out(1) + out(2)) * (1.0f / 3.0f);
      }
      const int64_t o = (int64_t)i * 3 + c;
      e.resid[o] = e.beta >= 1.0f ? pred : e.resid_in[o] + e.beta * (pred - e.resid_in[o]);
    }
  }
}

}  // namespace
}  // namespace lbm
