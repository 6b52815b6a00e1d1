// Internal declarations shared by the gfx950 kernels and the host runtime of
// liblbm.so.  Not part of the public ABI (see include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/lbm.h"

namespace lbm {

// Wall modes, outlet modes: same values as the public enums.
enum : int { kWallFreeSlip = 0, kWallPeriodic = 1, kWallNebb = 2, kWallMovingBB = 3 };
enum : int { kOutletCopyAll = 0, kOutletCopyUnknown = 1 };

// Force partials of one step live in a ring of kRing steps; a reduction
// kernel folds them into the FP64 history every kRing steps (and at the end
// of every lbm_step call).
constexpr int kRing = 96;

// Node flags inside the cylinder rectangle: bit 0 = solid node; bit k
// (k = 1..8) = the pull source x - c_k of this fluid node is solid, so
// population k arrives by half-way (or interpolated) bounce-back instead of
// streaming.  With full-way bounce-back the bits only mark the links whose
// momentum the node books; every population streams.
constexpr uint16_t kSolid = 1;

struct Geometry {
  int nx, ny;
  // population k of node (x, y) is at k * plane + y * pitch + x; the host
  // interleaves rows (plane = one row padded to a multiple of 64 floats,
  // pitch = 9 * plane), the kernels only use the two strides
  int pitch;        // floats from one row to the next (multiple of 64)
  int64_t plane;    // floats from one population to the next (multiple of 64)
  // cylinder rectangle [rx0, rx0+rw) x [ry0, ry0+rh) holding all solid nodes
  // and all their fluid neighbours; empty (rw = rh = 0) without a cylinder
  int rx0, ry0, rw, rh;
  const uint16_t* flags;  // [rh][rw]
  // [rh][rw]: position of a fluid node with bounce-back links in the list of
  // such nodes (row-major order), -1 elsewhere; fixes where each node's FP64
  // force contribution goes, so the sum order never depends on the tiling
  const int32_t* link_index;
  int n_link_nodes;
  // interpolated bounce-back: wall fraction q of the link of pull direction
  // k (1..8) of link node i at q[8 i + k - 1] (the link from the node along
  // -c_k ends in the solid); null with half-way bounce-back
  const float* q;
};

// Floats of one state buffer: the last population's last row ends there.
inline int64_t state_floats(const Geometry& g) { return 8 * g.plane + (int64_t)g.ny * g.pitch; }

struct Physics {
  float omega;     // 1/tau
  float u_in;      // inlet velocity
  float u_top, u_bot;
  int wall, outlet_mode, x_periodic;
  int mrt;         // 1: Eq. 6 with the rates below instead of Eq. 2
  int interp_bb;   // 1: interpolated bounce-back on the cylinder (Geometry::q)
  int full_bb;     // 1: full-way bounce-back: solid nodes stream and reverse
  float s_e, s_eps, s_qx, s_qy, s_pxx, s_pxy;  // rates of the non-conserved moments
};

// Tiling of one launch.  A tile is tile_x consecutive nodes of tile_y
// consecutive rows, handled by one block of 256 threads.
struct Tiling {
  int tile_x, tile_y;
  int ntx, nty;          // tiles along x and y
  int remap_xcd;         // block-to-tile map: 0 plain, 1 XCD bands, 2 XCD-interleaved rows
};

// Two to four steps per launch: each wave owns tile_x output columns (its
// 64 lanes hold one more column on either side per step beyond the first:
// kStrip2 = 62 for two steps, kStrip3 = 60 for three, kStrip4 = 58 for four)
// of one segment of tile_y rows.  Without x-periodicity the strips are aligned to the right
// edge.
constexpr int kStrip2 = 62;
constexpr int kStrip3 = 60;
constexpr int kStrip4 = 58;

__host__ __device__ inline int strip_halo(const Tiling& t) { return (64 - t.tile_x) / 2; }

__host__ __device__ inline int strip_start(const Geometry& g, const Tiling& t, bool x_periodic, int strip) {
  return x_periodic ? strip * t.tile_x : g.nx - t.tile_x * (t.ntx - strip);
}

// A segment is interior when it has the full tile_y rows and every node its
// wave updates in the first step (h = strip_halo columns and rows beyond the
// segment on every side) is plain bulk fluid: away from the edges and outside
// the cylinder's flag rectangle.  The others need the boundary code.
__host__ __device__ inline bool interior_segment(const Geometry& g, const Tiling& t, bool x_periodic, int strip,
                                                 int seg) {
  const int h = strip_halo(t);
  const int xs = strip_start(g, t, x_periodic, strip), y0 = seg * t.tile_y;
  const int xa = xs - h, xb = xs + t.tile_x - 1 + h, ya = y0 - h, yb = y0 + t.tile_y - 1 + h;
  if (xa < 1 || xb > g.nx - 2 || ya < 1 || yb > g.ny - 2) return false;
  return !(xa < g.rx0 + g.rw && xb >= g.rx0 && ya < g.ry0 + g.rh && yb >= g.ry0);
}

// One evaluation of the learned closure's network on the boundary nodes:
// nb nodes, the network's bfloat16 weights (Wb) and FP32 parameters
// (master), the feature normalisation and output scales (norm), the guards
// and filter, the residuals in use (resid_in) and the ones it writes.
struct ClosureEval {
  int blocks;  // in a step launch: the first `blocks` blocks evaluate the network (0: none)
  int nb, mask, taper, outlet_taper, outlet_neutral;
  float beta, limit;
  const uint16_t* Wb;
  const float* master;
  const float* norm;
  const float* bias;
  const float* resid_in;
  float* resid;
};

struct StepArgs {
  const float* __restrict__ A;  // post-collision populations f*(t), 9 planes
  float* __restrict__ B;        // receives f*(t+1)
  Geometry g;
  Physics p;
  Tiling t;
  double2* partial;             // this step's force contributions [n_link_nodes]
  double2* partial2;            // the second step's, for kernels that take two or three steps
  double2* partial3;            // the third step's, for kernels that take three or four
  double2* partial4;            // the fourth step's, for kernels that take four
  const int* gen;               // multi-step launches: segments (seg * ntx + strip) that are not interior
  int n_gen;
  const float* closure;         // learned-closure residuals [boundary node][3], or null
  int closure_mask;             // boundaries the closure refines: 1 top, 2 bottom, 4 outlet
  int* bad;                     // watchdog: min ring slot with a bad density
  int slot;                     // ring slot of this step
  ClosureEval ev;               // a network evaluation folded into the launch (two-step kernels)
};

// One case of an ensemble, as the batched kernels see it (device memory).
struct CaseArgs {
  float* buf[2];        // ping-pong population buffers (shifted storage)
  Geometry g;
  Physics p;
  Tiling t;             // one-step tiling (remap_xcd must be 0)
  Tiling tm;            // multi-step tiling of the ensemble's variant
  double2* partial;     // slot 0 of this case's force contributions; step j
                        // of the ring at partial + j * partial_stride
  int* bad;             // watchdog slot of this case
  int64_t* bad_step;    // first diverged step of this case (0 = none)
  int64_t* dev_step;    // steps folded into this case's history so far
  double* hist;         // [hist_cap][2] FP64 force history
  int64_t hist_cap;
};

struct Variant {
  const char* name;
  int tile_x, tile_y;  // nodes along x (= 256 * vx) and rows per tile; for two-step
                       // variants the output columns per wave and rows per segment
  int vx;              // consecutive nodes per lane on the bulk path
  int remap_xcd, nontemporal;
  int steps;           // time steps per launch (1, or 2-4 with the intermediate states in registers)
  int sub;             // two-step: rows per wave of the segments that need the boundary code
  int unrolled;        // 1: those waves issue every row's loads first, with no row loop
  int stream;          // multi-step: > 0 for interior waves that store each output row as it is
                       // made, loading this many rows ahead (bulk_wave_s); 0 holds them to the end
};

// Kernel launchers (lbm_kernels.hip).  All return the launch status.
int num_variants();
const Variant& variant(int v);  // 1-based
int default_variant(int64_t nodes);
hipError_t launch_step(const StepArgs& a, int v, hipStream_t s);
hipError_t launch_step_batch(const CaseArgs* cases, const int2* tiles, int ntiles, int cur, int slot,
                             int partial_stride, int v, hipStream_t s);
// Multi-step ensemble launch: boundary tasks first, then interior tasks
// (see multistep_batch_kernel); only variants multistep_batch_supported.
bool multistep_batch_supported(int v);
hipError_t launch_multistep_batch(const CaseArgs* cases, const int2* gen_tasks, int n_gen, const int2* bulk_tasks,
                                  int n_bulk, int cur, int slot, int partial_stride, int v, hipStream_t s);
hipError_t launch_force_reduce_batch(const CaseArgs* cases, int ncases, int count, int partial_stride,
                                     hipStream_t s);
hipError_t launch_force_reduce(const double2* partials, int nnodes, int count, double* hist,
                               int64_t cap, int64_t* dev_step, int* bad, int64_t* bad_step,
                               hipStream_t s);
hipError_t launch_init_equilibrium(float* f, const Geometry& g, double u, double amp, bool rest_solid,
                                   hipStream_t s);
hipError_t launch_fields(const float* f, const Geometry& g, float* rho, float* ux, float* uy,
                         hipStream_t s);
// dense [9][ny][nx] <-> pitched planes, with dtype 0 = f32, 1 = f64
hipError_t launch_pack(const float* f, const Geometry& g, void* dense, int dtype, hipStream_t s);
hipError_t launch_unpack(const void* dense, int dtype, const Geometry& g, float* f,
                         hipStream_t s);
hipError_t launch_fill_int(int* p, int value, hipStream_t s);
hipError_t launch_copy_probe(void* dst, const void* src, int64_t nbytes, hipStream_t s);

// learned closure (lbm_closure.hip)
constexpr int kMlpParams = 6723;
constexpr int kMlpBf16 = 48 * 64 + 64 * 64 + 64 * 16;  // padded bfloat16 weight copies
constexpr int kClosureNorm = 75;                      // mean[36], 1/std[36], out scale[3]
int mlp_blocks(int64_t B);
hipError_t launch_mlp_train(const float* X, const float* T, const int* idx, int B, const uint16_t* Wb,
                            const float* master, const float* norm, float* gpart, double* lpart, float noise,
                            uint64_t key, hipStream_t s);
hipError_t launch_mlp_adam(const float* gpart, int nblk, const double* lpart, float* master, float* m, float* v,
                           uint16_t* Wb, float* grad_out, double* loss_out, int step, float lr,
                           double inv_count, hipStream_t s);
hipError_t launch_mlp_forward(const float* X, int M, const uint16_t* Wb, const float* master, const float* norm,
                              float* Y, hipStream_t s);
hipError_t launch_sample_boundary(const float* A, const Geometry& g, int ox, int oy, int wnx, int wny,
                                  const int* nodes, int n, const float* bias, float* feat, float* target,
                                  hipStream_t s);
hipError_t launch_closure(const float* A, const Geometry& g, const ClosureEval& e, hipStream_t s);
int closure_blocks(int nb);     // blocks of one evaluation
size_t closure_lds_bytes();     // LDS of one evaluation block
// Whether a launch of k steps of variant v evaluates the network itself
// (StepArgs::ev) rather than after a closure_kernel launch.
bool step_fuses_closure(int v, int k);
hipError_t launch_column_moments(const float* X, int64_t M, int ncols, double* out, hipStream_t s);

// device weights of an lbm_mlp (lbm_closure_api.cpp)
struct MlpDevice {
  const uint16_t* Wb;
  const float* master;
};
MlpDevice mlp_device(const lbm_mlp* m);

// ------------------------------------------------------- host helpers
// (lbm_api.cpp) shared by the single-lattice and the ensemble runtimes.
struct HostGeometry {
  Geometry g;                       // device pointers left null
  std::vector<uint16_t> flags;      // [rh][rw]
  std::vector<int32_t> link_index;  // [rh][rw]
  std::vector<float> q;             // [n_link_nodes][8], interpolated bounce-back only
};
lbm_status build_geometry(const lbm_params* p, HostGeometry* out);
Physics make_physics(const lbm_params* p);
void tiling_for_variant(const Geometry& g, int v, Tiling* t);
lbm_status set_error(lbm_status s, const char* msg);

}  // namespace lbm
