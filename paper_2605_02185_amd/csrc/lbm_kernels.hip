// gfx950 kernels of the D2Q9 BGK cylinder-flow solver (arXiv 2605.02185).
//
// State between steps: post-collision populations f*(x, t) in 9 SoA planes,
// rows padded to a multiple of 64 floats.  One launch of step_kernel turns
// buffer A = f*(t) into buffer B = f*(t+1) node by node:
//   1. pull: f_k(x) = f*_k(x - c_k)                               (Eq. 2, LHS)
//      half-way bounce-back where x - c_k is solid: f_k(x) = f*_opp(k)(x)
//   2. boundary corrections of the populations missing at the edges
//      (Sec. 2.3: free-slip Eq. 7, periodic Eq. 8, NEBB Eqs. 9-10, moving-wall
//      bounce-back Eq. 11; outlet Eq. 13; Zou-He velocity inlet, Sec. 3.1)
//   3. moments (Eq. 4), equilibrium (Eq. 3), BGK relaxation (Eq. 2)
// The paper's order is collide -> stream -> correct; pulling the previous
// step's post-collision values and colliding at the end of the same pass is
// the same sequence shifted by half a step, with one read and one write of
// every population per step.
//
// Waves whose 64 nodes are all interior fluid nodes away from the cylinder
// take a branch-free bulk path; any other wave takes the general path, which
// looks the cylinder's bounce-back links up in a small flag rectangle.
#include "lbm_internal.h"

#include <climits>

namespace lbm {
namespace {

// Table 1 with k = i - 1, and the opposite directions.
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float W0 = 4.0f / 9.0f, W1 = 1.0f / 9.0f, W2 = 1.0f / 36.0f;

// Eq. 4 then Eqs. 2-3 on the nine streamed and corrected populations g;
// writes f* to B at element offset o of each plane.  Flags a density that is
// non-finite or outside (0, 10).
template <bool NT>
__device__ __forceinline__ void collide_store(const float (&g)[9], float omega, float* __restrict__ B,
                                              uint32_t plane, uint32_t o, bool& bad) {
  const float rho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  const float ir = 1.0f / rho;
  const float ux = (((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6])) * ir;
  const float uy = (((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8])) * ir;
  const float usq = 1.5f * (ux * ux + uy * uy);
  bad |= !(rho > 0.0f && rho < 10.0f);
  float cu[9];
  cu[0] = 0.0f;
  cu[1] = ux;
  cu[2] = uy;
  cu[3] = -ux;
  cu[4] = -uy;
  cu[5] = ux + uy;
  cu[6] = uy - ux;
  cu[7] = -(ux + uy);
  cu[8] = ux - uy;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float w = k == 0 ? W0 : (k < 5 ? W1 : W2);
    const float feq = w * rho * (1.0f - usq + cu[k] * (3.0f + 4.5f * cu[k]));
    const float v = g[k] + omega * (feq - g[k]);
    float* dst = B + k * plane + o;
    if (NT)
      __builtin_nontemporal_store(v, dst);
    else
      *dst = v;
  }
}

__device__ __forceinline__ uint16_t node_flags(const Geometry& g, int x, int y) {
  const unsigned rx = (unsigned)(x - g.rx0), ry = (unsigned)(y - g.ry0);
  if (rx < (unsigned)g.rw && ry < (unsigned)g.rh) return g.flags[ry * g.rw + rx];
  return 0;
}

__device__ __forceinline__ bool in_rect(const Geometry& g, int x, int y) {
  return (unsigned)(x - g.rx0) < (unsigned)g.rw && (unsigned)(y - g.ry0) < (unsigned)g.rh;
}

__device__ __forceinline__ float load(const float* __restrict__ A, const Geometry& g, int k, int x,
                                      int y) {
  return A[(uint32_t)k * (uint32_t)g.plane + (uint32_t)y * (uint32_t)g.pitch + (uint32_t)x];
}

// Streamed populations of node (x, y): pull with the wrap-arounds of the
// periodic modes and half-way bounce-back on the cylinder.  Populations
// whose source lies outside the lattice are the missing ones of Fig. 2; they
// are set to 0 here and overwritten by the boundary corrections.
__device__ __forceinline__ void pull(const StepArgs& a, int x, int y, uint16_t fl, float (&g)[9]) {
  const int nx = a.g.nx, ny = a.g.ny;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k > 0 && ((fl >> k) & 1)) {
      g[k] = load(a.A, a.g, OPP[k], x, y);
      continue;
    }
    int sx = x - CX[k], sy = y - CY[k];
    if (a.p.x_periodic) sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    if (a.p.wall == kWallPeriodic) sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    g[k] = (sx >= 0 && sx < nx && sy >= 0 && sy < ny) ? load(a.A, a.g, k, sx, sy) : 0.0f;
  }
}

// Top (y = ny-1) or bottom (y = 0) row correction at node (x, y).
__device__ __forceinline__ void wall_bc(const StepArgs& a, int x, int y, float (&g)[9]) {
  const bool top = y == a.g.ny - 1;
  switch (a.p.wall) {
    case kWallFreeSlip:  // Eq. 7: specular reflection at the node
      if (top) {
        g[4] = g[2];
        g[7] = g[6];
        g[8] = g[5];
      } else {
        g[2] = g[4];
        g[6] = g[7];
        g[5] = g[8];
      }
      break;
    case kWallNebb: {  // Eqs. 9-10: wall density from the known populations
      const float U = top ? a.p.u_top : a.p.u_bot;
      const float d13 = 0.5f * (g[1] - g[3]);
      if (top) {
        const float rw = (g[0] + g[1] + g[3]) + 2.0f * (g[2] + g[5] + g[6]);
        const float m = 0.5f * rw * U;
        g[4] = g[2];
        g[7] = g[5] + d13 - m;
        g[8] = g[6] - d13 + m;
      } else {
        const float rw = (g[0] + g[1] + g[3]) + 2.0f * (g[4] + g[7] + g[8]);
        const float m = 0.5f * rw * U;
        g[2] = g[4];
        g[5] = g[7] - d13 + m;
        g[6] = g[8] + d13 - m;
      }
      break;
    }
    case kWallMovingBB: {  // Eq. 11 with the node's own f* and density
      const float U = top ? a.p.u_top : a.p.u_bot;
      float fs[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) fs[k] = load(a.A, a.g, k, x, y);
      const float rho = ((fs[0] + fs[1]) + (fs[2] + fs[3])) + ((fs[4] + fs[5]) + (fs[6] + fs[7])) + fs[8];
      const float m = rho * U * (1.0f / 6.0f);
      if (top) {
        g[4] = fs[2];
        g[7] = fs[5] - m;
        g[8] = fs[6] + m;
      } else {
        g[2] = fs[4];
        g[5] = fs[7] + m;
        g[6] = fs[8] - m;
      }
      break;
    }
    default:
      break;
  }
}

// Streamed and row-corrected populations of node (x, y).
__device__ __forceinline__ void gather(const StepArgs& a, int x, int y, uint16_t fl, float (&g)[9]) {
  pull(a, x, y, fl, g);
  const bool wall_row = a.p.wall != kWallPeriodic && (y == 0 || y == a.g.ny - 1);
  const bool wall_x = a.p.x_periodic || (x >= 1 && x <= a.g.nx - 2);
  if (wall_row && wall_x) wall_bc(a, x, y, g);
}

template <bool NT>
__device__ __forceinline__ void general_node(const StepArgs& a, int x, int y, double& Fx, double& Fy,
                                          bool& bad) {
  const int nx = a.g.nx, ny = a.g.ny;
  const uint32_t o = (uint32_t)y * (uint32_t)a.g.pitch + (uint32_t)x;
  const uint32_t P = (uint32_t)a.g.plane;
  const bool open_x = !a.p.x_periodic;
  const bool outlet = open_x && x == nx - 1;
  const bool corner_y = a.p.wall != kWallPeriodic && (y == 0 || y == ny - 1);
  const uint16_t fl = node_flags(a.g, x, y);
  if (fl & kSolid) {  // solid nodes keep their (never streamed) values
#pragma unroll
    for (int k = 0; k < 9; ++k) a.B[k * P + o] = a.A[k * P + o];
    return;
  }
  float g[9];
  if (outlet) {
    // Eq. 13: the outlet column takes the corrected populations of x = nx-2
    gather(a, nx - 2, y, node_flags(a.g, nx - 2, y), g);
    if (a.p.outlet_mode == kOutletCopyUnknown && !corner_y) {
      float own[9];
      pull(a, x, y, fl, own);
      g[0] = own[0];
      g[1] = own[1];
      g[2] = own[2];
      g[4] = own[4];
      g[5] = own[5];
      g[8] = own[8];
    }
  } else {
    gather(a, x, y, fl, g);
  }
  if (open_x && x == 0) {
    const float U = a.p.u_in;
    if (corner_y) {  // inlet corners: equilibrium at rho = 1, u = (U, 0)
      const float usq = 1.5f * U * U;
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float w = k == 0 ? W0 : (k < 5 ? W1 : W2);
        const float cu = (float)CX[k] * U;
        g[k] = w * (1.0f - usq + cu * (3.0f + 4.5f * cu));
      }
    } else {  // Zou-He velocity inlet, u = (U, 0)
      const float rho = ((g[0] + g[2]) + g[4] + 2.0f * ((g[3] + g[6]) + g[7])) / (1.0f - U);
      const float d24 = 0.5f * (g[2] - g[4]);
      g[1] = g[3] + (2.0f / 3.0f) * rho * U;
      g[5] = g[7] - d24 + rho * U * (1.0f / 6.0f);
      g[8] = g[6] + d24 + rho * U * (1.0f / 6.0f);
    }
  }
  if (fl >> 1) {
    // Eq. 14: each bounced population g_k = f*_opp(k)(x) left along c_opp(k)
    // and came back along c_k, giving the body 2 c_opp(k) f*_opp(k).
#pragma unroll
    for (int k = 1; k < 9; ++k)
      if ((fl >> k) & 1) {
        Fx -= 2.0 * (double)CX[k] * (double)g[k];
        Fy -= 2.0 * (double)CY[k] * (double)g[k];
      }
  }
  collide_store<NT>(g, a.p.omega, a.B, P, o, bad);
}

template <bool NT>
__device__ __forceinline__ void bulk_node(const StepArgs& a, int x, int y, bool& bad) {
  const float* __restrict__ A = a.A;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
  const uint32_t o = (uint32_t)y * Wp + (uint32_t)x;
  float g[9];
  g[0] = A[o];
  g[1] = A[P + o - 1];
  g[2] = A[2 * P + o - Wp];
  g[3] = A[3 * P + o + 1];
  g[4] = A[4 * P + o + Wp];
  g[5] = A[5 * P + o - Wp - 1];
  g[6] = A[6 * P + o - Wp + 1];
  g[7] = A[7 * P + o + Wp + 1];
  g[8] = A[8 * P + o + Wp - 1];
  collide_store<NT>(g, a.p.omega, a.B, P, o, bad);
}

// Blocks are dispatched round-robin over the 8 XCDs (block id mod 8); hand
// each XCD a contiguous range of tiles so that neighbouring tiles, which
// share halo cache lines, meet in the same L2.
__device__ __forceinline__ int remap_xcd(int id, int n) {
  const int xcd = id & 7, local = id >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + min(xcd, rem) + local;
}

// FP64 sum of (fx, fy) over the block; thread 0 gets the result.
__device__ __forceinline__ double2 block_sum(double fx, double fy) {
  __shared__ double2 part[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    fx += __shfl_xor(fx, off);
    fy += __shfl_xor(fy, off);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) part[wave] = make_double2(fx, fy);
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      s.x += part[w].x;
      s.y += part[w].y;
    }
  return s;
}

template <int TY, bool NT>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a) {
  const int ntiles = a.t.ntx * a.t.nty;
  const int tile = a.t.remap_xcd ? remap_xcd((int)blockIdx.x, ntiles) : (int)blockIdx.x;
  const int bx = tile % a.t.ntx, by = tile / a.t.ntx;
  const int nx = a.g.nx, ny = a.g.ny;
  const int x = bx * a.t.tile_x + (int)threadIdx.x;
  double Fx = 0.0, Fy = 0.0;
  bool bad = false;
#pragma unroll
  for (int r = 0; r < TY; ++r) {
    const int y = by * TY + r;
    const bool active = x < nx && y < ny;
    const bool special =
        active && (x == 0 || x == nx - 1 || y == 0 || y == ny - 1 || in_rect(a.g, x, y));
    if (__any(special)) {
      if (active) general_node<NT>(a, x, y, Fx, Fy, bad);
    } else if (active) {
      bulk_node<NT>(a, x, y, bad);
    }
  }
  if (bad) atomicMin(a.bad, a.slot);
  const unsigned fxr = (unsigned)(bx - a.t.fx0), fyr = (unsigned)(by - a.t.fy0);
  if (fxr < (unsigned)a.t.fw && fyr < (unsigned)a.t.fh) {
    const double2 s = block_sum(Fx, Fy);
    if (threadIdx.x == 0) a.partial[fyr * a.t.fw + fxr] = s;
  }
}

// Folds `count` rows of force partials into the FP64 history in a fixed
// order, advances the device step counter and converts the watchdog slot
// into an absolute step.  One block.
__global__ __launch_bounds__(256) void force_reduce_kernel(const double2* __restrict__ partials,
                                                           int nslots, int count, double* hist,
                                                           int64_t cap, int64_t* dev_step, int* bad,
                                                           int64_t* bad_step) {
  __shared__ double2 sh[256];
  const int64_t base = *dev_step;
  for (int j = 0; j < count; ++j) {
    double sx = 0.0, sy = 0.0;
    for (int i = threadIdx.x; i < nslots; i += 256) {
      const double2 v = partials[(int64_t)j * nslots + i];
      sx += v.x;
      sy += v.y;
    }
    sh[threadIdx.x] = make_double2(sx, sy);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) {
        sh[threadIdx.x].x += sh[threadIdx.x + w].x;
        sh[threadIdx.x].y += sh[threadIdx.x + w].y;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const int64_t s = (base + j) % cap;
      hist[2 * s] = sh[0].x;
      hist[2 * s + 1] = sh[0].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int b = *bad;
    if (b != INT_MAX) {
      if (*bad_step == 0) *bad_step = base + b + 1;
      *bad = INT_MAX;
    }
    *dev_step = base + count;
  }
}

__global__ void init_eq_kernel(float* f, Geometry g, double u, double amp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  const double v = amp * u * sin(2.0 * 3.14159265358979323846 * y / (double)(g.ny - 1));
  const double usq = 1.5 * (u * u + v * v);
  for (int k = 0; k < 9; ++k) {
    const double w = k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    const double cu = CX[k] * u + CY[k] * v;
    f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x] = (float)(w * (1.0 - usq + cu * (3.0 + 4.5 * cu)));
  }
}

__global__ void fields_kernel(const float* __restrict__ f, Geometry g, float* rho, float* ux, float* uy) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = (int64_t)y * g.nx + x;
  float r = 1.0f, u = 0.0f, v = 0.0f;
  if (!(node_flags(g, x, y) & kSolid)) {
    float h[9];
    for (int k = 0; k < 9; ++k) h[k] = f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x];
    r = ((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8];
    u = (((h[1] - h[3]) + (h[5] - h[7])) + (h[8] - h[6])) / r;
    v = (((h[2] - h[4]) + (h[5] - h[7])) + (h[6] - h[8])) / r;
  }
  if (rho) rho[i] = r;
  if (ux) ux[i] = u;
  if (uy) uy[i] = v;
}

__global__ void pack_kernel(const float* __restrict__ f, Geometry g, void* dense, int dtype) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const float v = f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x];
  const int64_t i = ((int64_t)k * g.ny + y) * g.nx + x;
  if (dtype == 0)
    ((float*)dense)[i] = v;
  else
    ((double*)dense)[i] = (double)v;
}

__global__ void unpack_kernel(const void* dense, int dtype, Geometry g, float* f) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = ((int64_t)k * g.ny + y) * g.nx + x;
  const float v = dtype == 0 ? ((const float*)dense)[i] : (float)((const double*)dense)[i];
  f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x] = v;
}

__global__ void fill_int_kernel(int* p, int value) { *p = value; }

constexpr Variant kVariants[] = {
    {"tx256_ty1_xcd_nt", 256, 1, 1, 1},
    {"tx256_ty1_nt", 256, 1, 0, 1},
    {"tx256_ty1_xcd", 256, 1, 1, 0},
    {"tx256_ty2_xcd_nt", 256, 2, 1, 1},
    {"tx256_ty4_xcd_nt", 256, 4, 1, 1},
};

}  // namespace

int num_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const Variant& variant(int v) { return kVariants[v - 1]; }

hipError_t launch_step(const StepArgs& a, int v, hipStream_t s) {
  const Variant& var = variant(v);
  const dim3 grid((unsigned)(a.t.ntx * a.t.nty)), block((unsigned)var.tile_x);
  if (var.tile_y == 1) {
    if (var.nontemporal)
      hipLaunchKernelGGL((step_kernel<1, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((step_kernel<1, false>), grid, block, 0, s, a);
  } else if (var.tile_y == 2) {
    hipLaunchKernelGGL((step_kernel<2, true>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((step_kernel<4, true>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_force_reduce(const double2* partials, int nslots, int count, double* hist,
                               int64_t cap, int64_t* dev_step, int* bad, int64_t* bad_step,
                               hipStream_t s) {
  hipLaunchKernelGGL(force_reduce_kernel, dim3(1), dim3(256), 0, s, partials, nslots, count, hist,
                     cap, dev_step, bad, bad_step);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(float* f, const Geometry& g, double u, double amp, hipStream_t s) {
  hipLaunchKernelGGL(init_eq_kernel, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, f, g, u, amp);
  return hipGetLastError();
}

hipError_t launch_fields(const float* f, const Geometry& g, float* rho, float* ux, float* uy,
                         hipStream_t s) {
  hipLaunchKernelGGL(fields_kernel, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, f, g, rho, ux, uy);
  return hipGetLastError();
}

hipError_t launch_pack(const float* f, const Geometry& g, void* dense, int dtype, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3((g.nx + 255) / 256, g.ny, 9), dim3(256), 0, s, f, g, dense, dtype);
  return hipGetLastError();
}

hipError_t launch_unpack(const void* dense, int dtype, const Geometry& g, float* f, hipStream_t s) {
  hipLaunchKernelGGL(unpack_kernel, dim3((g.nx + 255) / 256, g.ny, 9), dim3(256), 0, s, dense, dtype, g, f);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int value, hipStream_t s) {
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, s, p, value);
  return hipGetLastError();
}

}  // namespace lbm
