// gfx950 kernels of the D2Q9 lattice Boltzmann cylinder-flow solver (arXiv 2605.02185).
//
// State between steps: post-collision populations f*(x, t), each row of the
// lattice holding the nine populations' rows one after another (structure of
// arrays within a row), rows padded to a multiple of 64 floats, stored
// shifted by the rest
// equilibrium as h_k = f*_k - w_k (FP32).  The deviations are two orders of
// magnitude smaller than f itself, so FP32 rounding errors shrink by the same
// factor (shifted storage, Skordos 1993).  Every population formula of the
// boundary treatments pairs directions of equal weight, so it reads the same
// on h as on f; only densities carry the explicit 1 = sum of the weights.  One launch of step_kernel turns
// buffer A = f*(t) into buffer B = f*(t+1) node by node:
//   1. pull: f_k(x) = f*_k(x - c_k)                               (Eq. 2, LHS)
//      half-way bounce-back where x - c_k is solid: f_k(x) = f*_opp(k)(x)
//      (or interpolated bounce-back, Sec. 2.4, or full-way, Sec. 3.1)
//   2. boundary corrections of the populations missing at the edges
//      (Sec. 2.3: free-slip Eq. 7, periodic Eq. 8, NEBB Eqs. 9-10, moving-wall
//      bounce-back Eq. 11; outlet Eq. 13; Zou-He velocity inlet, Sec. 3.1)
//   3. moments (Eq. 4), equilibrium (Eq. 3), BGK relaxation (Eq. 2) or the
//      multiple-relaxation-time collision of Eq. 6
// The paper's order is collide -> stream -> correct; pulling the previous
// step's post-collision values and colliding at the end of the same pass is
// the same sequence shifted by half a step, with one read and one write of
// every population per step.
//
// Waves whose 64 nodes are all interior fluid nodes away from the cylinder
// take a branch-free bulk path; any other wave takes the general path, which
// looks the cylinder's bounce-back links up in a small flag rectangle.
//
// step2_kernel and multistep_kernel take the same per-node steps two, three
// or four times in one launch (temporal blocking): each wave keeps the
// intermediate levels f*(t+1) .. f*(t+S-1) of a strip of columns in
// registers, reaching x-neighbours by DPP lane shifts, recomputes one more
// column and row on every side per level, and stores only f*(t+S).  Every
// variant gives the same bits as one step per launch.
#include "lbm_internal.h"
#include "lbm_mlp_dev.h"

#include <climits>
#include <cstring>

namespace lbm {
namespace {

// Table 1 with k = i - 1, and the opposite directions.
constexpr int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr float W0 = 4.0f / 9.0f, W1 = 1.0f / 9.0f, W2 = 1.0f / 36.0f;

// Eq. 4 then Eqs. 2-3 on the nine streamed and corrected deviations
// g_k = f_k - w_k, giving the post-collision deviations out.  With
// drho = rho - 1 = sum g_k and j = sum c_k g_k:
//   f_eq,k - w_k = w_k [drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)],
// and the relaxation g + omega (f_eq - w - g) is formed as
// (1 - omega) g + (omega w) [drho + rho (...)], one instruction fewer per
// population (the factors are uniform across the wave).  Contraction is off
// and every fused multiply-add is written out, so that each kernel variant
// (scalar or vector bulk path, general path) rounds identically.
__device__ __forceinline__ void collide_bgk(const float (&g)[9], float drho, float rho, float ux, float uy,
                                            float omega, float (&out)[9]) {
#pragma clang fp contract(off)
  const float keep = 1.0f - omega;
  const float usq = 1.5f * __fmaf_rn(ux, ux, uy * uy);
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
    const float ow = omega * (k == 0 ? W0 : (k < 5 ? W1 : W2));
    const float poly = __fmaf_rn(cu[k], __fmaf_rn(4.5f, cu[k], 3.0f), -usq);
    out[k] = __fmaf_rn(keep, g[k], ow * __fmaf_rn(rho, poly, drho));
  }
}

// Eq. 6: f* = f - M^-1 S (M f - m_eq), on the deviations g.  The rows of M
// are orthogonal, M M^T = D = diag(9, 36, 36, 6, 12, 6, 12, 4, 4), so
// M^-1 = M^T D^-1 and the correction of population k is
//   sum_i M_ik a_i,   a_i = s_i (m_i - m_eq,i) / D_i,
// over the six non-conserved moments (rho, j_x, j_y are unchanged because
// their equilibria equal them).  The rest state's moments M w are
// (1, -2, 1, 0, ...), so m - m_eq is formed from the moments of g and
// drho, j without cancellation of O(1) terms:
//   e:   M_e g + 2 drho - 3 rho u.u      eps: M_eps g - drho + 3 rho u.u
//   q_x: M_qx g + j_x                    q_y: M_qy g + j_y
//   p_xx: M_pxx g - rho (u_x^2 - u_y^2)  p_xy: M_pxy g - rho u_x u_y
// with m_eq = rho (-2 + 3 u.u, 1 - 3 u.u, u_x, -u_x, u_y, -u_y,
// u_x^2 - u_y^2, u_x u_y), the equilibrium moments of Eq. 3.
//
// All moments come from eight sums and differences of opposite pairs
// (a13 = g1 + g3, d13 = g1 - g3, ...): rho - 1 = g0 + s14 + s58,
// j_x = d13 + (d57 + d86), j_y = d24 + (d57 - d86), M_qx g = -2 d13 + (d57 +
// d86), M_qy g = -2 d24 + (d57 - d86), M_pxx g = a13 - a24, M_pxy g = a57 -
// a68, with s14 = a13 + a24 and s58 = a57 + a68 in M_e g and M_eps g.  The
// node's moments and the density check are done here (collide_t calls it
// for MRT before computing the BGK path's own sums).
__device__ __forceinline__ void collide_mrt(const float (&g)[9], const Physics& p, float (&out)[9], bool& bad) {
#pragma clang fp contract(off)
  const float a13 = g[1] + g[3], a24 = g[2] + g[4], a57 = g[5] + g[7], a68 = g[6] + g[8];
  const float d13 = g[1] - g[3], d24 = g[2] - g[4], d57 = g[5] - g[7], d86 = g[8] - g[6];
  const float s14 = a13 + a24, s58 = a57 + a68;
  const float e = d57 + d86, f = d57 - d86;
  const float drho = (g[0] + s14) + s58;
  const float rho = 1.0f + drho;
  const float ir = __builtin_amdgcn_rcpf(rho);
  const float jx = d13 + e;
  const float jy = d24 + f;
  const float ux = jx * ir;
  const float uy = jy * ir;
  bad |= !(rho > 0.0f && rho < 10.0f);
  const float ru2 = rho * __fmaf_rn(ux, ux, uy * uy);
  const float me = __fmaf_rn(2.0f, s58, __fmaf_rn(-4.0f, g[0], -s14));
  const float meps = __fmaf_rn(-2.0f, s14, __fmaf_rn(4.0f, g[0], s58));
  const float mqx = __fmaf_rn(-2.0f, d13, e);
  const float mqy = __fmaf_rn(-2.0f, d24, f);
  const float mpxx = a13 - a24;
  const float mpxy = a57 - a68;
  const float a1 = p.s_e * (1.0f / 36.0f) * __fmaf_rn(-3.0f, ru2, __fmaf_rn(2.0f, drho, me));
  const float a2 = p.s_eps * (1.0f / 36.0f) * __fmaf_rn(3.0f, ru2, meps - drho);
  const float a4 = p.s_qx * (1.0f / 12.0f) * (mqx + jx);
  const float a6 = p.s_qy * (1.0f / 12.0f) * (mqy + jy);
  const float a7 = p.s_pxx * 0.25f * __fmaf_rn(-rho, __fmaf_rn(ux, ux, -(uy * uy)), mpxx);
  const float a8 = p.s_pxy * 0.25f * __fmaf_rn(-rho, ux * uy, mpxy);
  // columns of M: rest (1,-4,4,...), axis k (1,-1,-2, c_x, -2c_x, c_y, -2c_y,
  // c_x^2-c_y^2, 0), diagonal k (1,2,1, c_x, c_x, c_y, c_y, 0, c_x c_y)
  const float axis = __fmaf_rn(2.0f, a2, a1);
  const float diag = __fmaf_rn(2.0f, a1, a2);
  out[0] = __fmaf_rn(4.0f, a1 - a2, g[0]);
  out[1] = g[1] + (__fmaf_rn(2.0f, a4, axis) - a7);
  out[2] = g[2] + (__fmaf_rn(2.0f, a6, axis) + a7);
  out[3] = g[3] + (__fmaf_rn(-2.0f, a4, axis) - a7);
  out[4] = g[4] + (__fmaf_rn(-2.0f, a6, axis) + a7);
  out[5] = g[5] - ((diag + a8) + (a4 + a6));
  out[6] = g[6] - ((diag - a8) + (a6 - a4));
  out[7] = g[7] - ((diag + a8) - (a4 + a6));
  out[8] = g[8] - ((diag - a8) + (a4 - a6));
}

// Moments (Eq. 4) and the collision.  1/rho is the hardware reciprocal
// (within 1 ulp): a correctly rounded division costs about ten instructions,
// a tenth of the whole collision.  COLL picks the operator at compile time
// (kBgk, kMrt) or from p.mrt (kEither); the arithmetic is the same either way.
enum : int { kBgk = 0, kMrt = 1, kEither = 2 };
template <int COLL>
__device__ __forceinline__ void collide_t(const float (&g)[9], const Physics& p, float (&out)[9], bool& bad) {
#pragma clang fp contract(off)
  if (COLL == kMrt || (COLL == kEither && p.mrt)) {
    collide_mrt(g, p, out, bad);
    return;
  }
  const float drho = ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])) + g[8];
  const float rho = 1.0f + drho;
  const float ir = __builtin_amdgcn_rcpf(rho);
  const float jx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
  const float jy = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
  const float ux = jx * ir;
  const float uy = jy * ir;
  bad |= !(rho > 0.0f && rho < 10.0f);
  collide_bgk(g, drho, rho, ux, uy, p.omega, out);
}

__device__ __forceinline__ void collide(const float (&g)[9], const Physics& p, float (&out)[9], bool& bad) {
  collide_t<kEither>(g, p, out, bad);
}

template <bool NT>
__device__ __forceinline__ void store9(float* __restrict__ B, uint32_t plane, uint32_t o, const float (&v)[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    float* dst = B + k * plane + o;
    if (NT)
      __builtin_nontemporal_store(v[k], dst);
    else
      *dst = v[k];
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

// Interpolated bounce-back (Sec. 2.4; the linear scheme of Bouzidi,
// Firdaouss & Lallemand) for the population arriving along c_k at a fluid
// node whose neighbour x - c_k is solid, the wall cutting that link at the
// fraction q: fo = f*_opp(k)(x) (what left towards the wall), fb =
// f*_opp(k)(x + c_k) (the same population one node further from the wall),
// fk = f*_k(x).  q < 1/2 interpolates 2q fo + (1 - 2q) fb, q >= 1/2
// interpolates fo / (2q) + (1 - 1/(2q)) fk; both give fo at q = 1/2.  The
// weights sum to one and opposite directions share a weight, so the same
// formula holds on the stored deviations f - w.
__device__ __forceinline__ float bfl(float q, float fo, float fb, float fk) {
#pragma clang fp contract(off)
  if (q < 0.5f) {
    const float t = 2.0f * q;
    return __fmaf_rn(t, fo, (1.0f - t) * fb);
  }
  const float r = 0.5f / q;
  return __fmaf_rn(r, fo, (1.0f - r) * fk);
}

__device__ __forceinline__ int link_slot(const Geometry& geo, int x, int y) {
  return geo.link_index[(y - geo.ry0) * geo.rw + (x - geo.rx0)];
}

// Streamed populations of node (x, y): pull with the wrap-arounds of the
// periodic modes and bounce-back on the cylinder (half-way, or interpolated
// with the links' wall fractions; with full-way bounce-back the solid
// neighbour's reversed populations stream in like any other).  Populations
// whose source lies outside the lattice are the missing ones of Fig. 2; they
// are set to 0 here and overwritten by the boundary corrections.
__device__ __forceinline__ void pull(const StepArgs& a, int x, int y, uint16_t fl, float (&g)[9]) {
  const int nx = a.g.nx, ny = a.g.ny;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    if (k > 0 && ((fl >> k) & 1) && !a.p.full_bb) {
      const float fo = load(a.A, a.g, OPP[k], x, y);
      if (a.p.interp_bb) {
        const float q = a.g.q[8 * link_slot(a.g, x, y) + k - 1];
        // the cylinder keeps two nodes from every edge: x + c_k is inside
        const float fb = q < 0.5f ? load(a.A, a.g, OPP[k], x + CX[k], y + CY[k]) : 0.0f;
        const float fk = q < 0.5f ? 0.0f : load(a.A, a.g, k, x, y);
        g[k] = bfl(q, fo, fb, fk);
      } else {
        g[k] = fo;
      }
      continue;
    }
    int sx = x - CX[k], sy = y - CY[k];
    if (a.p.x_periodic) sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    if (a.p.wall == kWallPeriodic) sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    g[k] = (sx >= 0 && sx < nx && sy >= 0 && sy < ny) ? load(a.A, a.g, k, sx, sy) : 0.0f;
  }
}

// Top (y = ny-1) or bottom (y = 0) row correction of the streamed
// populations g of one node; fs are the node's own post-collision
// populations f*(t), read only by the moving-wall treatment.
__device__ __forceinline__ void wall_bc(const Physics& p, bool top, const float (&fs)[9], float (&g)[9]) {
  // Both rows are written with selects: as two branches the compiler merges
  // them into run-time indexing of g, which moves g to scratch memory.  With
  // sg = +1 on the top row and -1 on the bottom row the sign flips are exact,
  // so each row gets the same arithmetic as its own formula.
  const float sg = top ? 1.0f : -1.0f;
  switch (p.wall) {
    case kWallFreeSlip: {  // Eq. 7: specular reflection at the node
      const float a2 = g[2], a4 = g[4], a5 = g[5], a6 = g[6], a7 = g[7], a8 = g[8];
      g[4] = top ? a2 : a4;  // top: S, SW, SE from N, NW, NE
      g[7] = top ? a6 : a7;
      g[8] = top ? a5 : a8;
      g[2] = top ? a2 : a4;  // bottom: N, NW, NE from S, SW, SE
      g[6] = top ? a6 : a7;
      g[5] = top ? a5 : a8;
      break;
    }
    case kWallNebb: {  // Eqs. 9-10: wall density from the known populations
      const float U = top ? p.u_top : p.u_bot;
      const float d13 = 0.5f * (g[1] - g[3]);
      // the populations leaving through the wall: N, NE, NW (top), S, SW, SE (bottom)
      const float k0 = top ? g[2] : g[4], k1 = top ? g[5] : g[7], k2 = top ? g[6] : g[8];
      const float rw = 1.0f + ((g[0] + g[1] + g[3]) + 2.0f * (k0 + k1 + k2));
      const float m = 0.5f * rw * U;
      const float n1 = (k1 + sg * d13) - sg * m, n2 = (k2 - sg * d13) + sg * m;
      g[4] = top ? k0 : g[4];
      g[7] = top ? n1 : g[7];
      g[8] = top ? n2 : g[8];
      g[2] = top ? g[2] : k0;
      g[5] = top ? g[5] : n1;
      g[6] = top ? g[6] : n2;
      break;
    }
    case kWallMovingBB: {  // Eq. 11 with the node's own f* and density
      const float U = top ? p.u_top : p.u_bot;
      const float rho = 1.0f + (((fs[0] + fs[1]) + (fs[2] + fs[3])) + ((fs[4] + fs[5]) + (fs[6] + fs[7])) + fs[8]);
      const float m = rho * U * (1.0f / 6.0f);
      const float k0 = top ? fs[2] : fs[4], k1 = top ? fs[5] : fs[7], k2 = top ? fs[6] : fs[8];
      const float n1 = k1 - sg * m, n2 = k2 + sg * m;
      g[4] = top ? k0 : g[4];
      g[7] = top ? n1 : g[7];
      g[8] = top ? n2 : g[8];
      g[2] = top ? g[2] : k0;
      g[5] = top ? g[5] : n1;
      g[6] = top ? g[6] : n2;
      break;
    }
    default:
      break;
  }
}

// Zou-He velocity inlet, u = (U, 0), on the streamed populations of an inlet
// node; the two inlet corners are equilibrium nodes at rho = 1, u = (U, 0).
__device__ __forceinline__ void inlet_bc(const Physics& p, bool corner, float (&g)[9]) {
  const float U = p.u_in;
  if (corner) {
    const float usq = 1.5f * U * U;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float w = k == 0 ? W0 : (k < 5 ? W1 : W2);
      const float cu = (float)CX[k] * U;
      g[k] = w * (cu * (3.0f + 4.5f * cu) - usq);
    }
  } else {  // the known weights sum to 1
    const float rho = (1.0f + ((g[0] + g[2]) + g[4] + 2.0f * ((g[3] + g[6]) + g[7]))) / (1.0f - U);
    const float d24 = 0.5f * (g[2] - g[4]);
    g[1] = g[3] + (2.0f / 3.0f) * rho * U;
    g[5] = g[7] - d24 + rho * U * (1.0f / 6.0f);
    g[8] = g[6] + d24 + rho * U * (1.0f / 6.0f);
  }
}

// Eq. 14: on each link the population f*_opp(k)(x) left along c_opp(k) and
// g_k came back along c_k, giving the body (f*_opp(k) + g_k) c_opp(k); with
// half-way bounce-back both are f*_opp(k): 2 c_opp(k) g_k.  With full-way
// bounce-back f*_opp(k)(x) enters the solid node now and comes back reversed
// one step later; its whole exchange, 2 c_opp(k) f*_opp(k)(x), is booked
// now.  `own` holds the node's post-collision f* (read by the interpolated
// and full-way modes).  Written to the node's fixed slot `li` of this step's
// contributions (its position in the list of link nodes).
__device__ __forceinline__ void link_force(double2* __restrict__ partial, int li, uint16_t fl, const float (&g)[9],
                                           const float (&own)[9], const Physics& p) {
  double Fx = 0.0, Fy = 0.0;
#pragma unroll
  for (int k = 1; k < 9; ++k)
    if ((fl >> k) & 1) {
      const double w = k < 5 ? 1.0 / 9.0 : 1.0 / 36.0;
      if (p.interp_bb) {
        const double sum = ((double)own[OPP[k]] + w) + ((double)g[k] + w);
        Fx -= (double)CX[k] * sum;
        Fy -= (double)CY[k] * sum;
      } else if (p.full_bb) {
        const double fo = (double)own[OPP[k]] + w;
        Fx -= 2.0 * (double)CX[k] * fo;
        Fy -= 2.0 * (double)CY[k] * fo;
      } else {
        const double fk = (double)g[k] + w;
        Fx -= 2.0 * (double)CX[k] * fk;
        Fy -= 2.0 * (double)CY[k] * fk;
      }
    }
  partial[li] = make_double2(Fx, Fy);
}

// Learned-closure residuals (when enabled) on the three missing populations
// of a wall-row node (top row nodes 0 .. nx-3, bottom row nodes nx-2 ..
// 2nx-5 of the closure's boundary numbering) and of an outlet node (nodes
// 2(nx-2) ..).
// (Selects rather than two branches: merged branches index g at run time,
// which moves g to scratch memory.)
__device__ __forceinline__ void closure_row(const StepArgs& a, int x, int y, float (&g)[9]) {
  if (!a.closure) return;
  const bool top = y == a.g.ny - 1;
  const float* r = a.closure + 3 * ((top ? 0 : a.g.nx - 2) + (x - 1));
  const float r0 = r[0], r1 = r[1], r2 = r[2];
  g[4] = top ? g[4] + r0 : g[4];
  g[7] = top ? g[7] + r1 : g[7];
  g[8] = top ? g[8] + r2 : g[8];
  g[2] = top ? g[2] : g[2] + r0;
  g[6] = top ? g[6] : g[6] + r1;
  g[5] = top ? g[5] : g[5] + r2;
}

// The same wall-row residuals as closure_row, taken from registers: rt and rb
// hold this lane's entries for the top and bottom rows (closure_rows_load).
__device__ __forceinline__ void closure_row_regs(const StepArgs& a, bool top, const float (&rt)[3],
                                                 const float (&rb)[3], float (&g)[9]) {
  if (!a.closure) return;
  const float r0 = top ? rt[0] : rb[0], r1 = top ? rt[1] : rb[1], r2 = top ? rt[2] : rb[2];
  g[4] = top ? g[4] + r0 : g[4];
  g[7] = top ? g[7] + r1 : g[7];
  g[8] = top ? g[8] + r2 : g[8];
  g[2] = top ? g[2] : g[2] + r0;
  g[6] = top ? g[6] : g[6] + r1;
  g[5] = top ? g[5] : g[5] + r2;
}

// Column x's residuals on the top and bottom rows, read when `need` (the
// caller's rows include a wall row); zeros without a closure.  Columns
// outside 1 .. nx-2, which have none, read column 1 or nx-2 and never apply
// them.
__device__ __forceinline__ void closure_rows_load(const StepArgs& a, bool need, int x, float (&rt)[3],
                                                  float (&rb)[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) rt[c] = rb[c] = 0.0f;
  if (!a.closure || !need) return;
  const int i = min(max(x, 1), a.g.nx - 2) - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    rt[c] = a.closure[3 * i + c];
    rb[c] = a.closure[3 * (a.g.nx - 2 + i) + c];
  }
}

__device__ __forceinline__ void closure_outlet(const StepArgs& a, int y, float (&g)[9]) {
  if (!a.closure || !(a.closure_mask & 4)) return;
  const float* r = a.closure + 3 * (2 * (a.g.nx - 2) + (y - 1));
  g[3] += r[0];
  g[6] += r[1];
  g[7] += r[2];
}

// Streamed and row-corrected populations of node (x, y).  With a learned
// closure the network's residuals are added to the wall treatment's values
// of the three missing populations (top row nodes 0 .. nx-3, bottom row
// nodes nx-2 .. 2nx-5 of the closure's boundary numbering).
__device__ __forceinline__ void gather(const StepArgs& a, int x, int y, uint16_t fl, float (&g)[9]) {
  pull(a, x, y, fl, g);
  const bool wall_row = a.p.wall != kWallPeriodic && (y == 0 || y == a.g.ny - 1);
  const bool wall_x = a.p.x_periodic || (x >= 1 && x <= a.g.nx - 2);
  if (wall_row && wall_x) {
    float fs[9];
    if (a.p.wall == kWallMovingBB) {
#pragma unroll
      for (int k = 0; k < 9; ++k) fs[k] = load(a.A, a.g, k, x, y);
    }
    wall_bc(a.p, y == a.g.ny - 1, fs, g);
    closure_row(a, x, y, g);
  }
}

// Post-collision populations f*(t+1) of a node that is not plain bulk
// fluid: pull, boundary corrections, force contributions (written when
// `owner`), collision.  Solid nodes keep their (never streamed) values, or
// with full-way bounce-back pull theirs and send them back reversed.
template <int COLL = kEither>
__device__ __forceinline__ void general_update(const StepArgs& a, int x, int y, bool owner, float (&out)[9],
                                               bool& bad) {
  const int nx = a.g.nx, ny = a.g.ny;
  const bool open_x = !a.p.x_periodic;
  const bool outlet = open_x && x == nx - 1;
  const bool corner_y = a.p.wall != kWallPeriodic && (y == 0 || y == ny - 1);
  const uint16_t fl = node_flags(a.g, x, y);
  if (fl & kSolid) {
    if (a.p.full_bb) {
      float g[9];
      pull(a, x, y, 0, g);
#pragma unroll
      for (int k = 0; k < 9; ++k) out[k] = g[OPP[k]];
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) out[k] = load(a.A, a.g, k, x, y);
    }
    return;
  }
  float g[9];
  if (outlet) {
    // Eq. 13: the outlet column takes the corrected populations of x = nx-2
    // (copy-all), or only those that stream in from outside the lattice
    // (copy-unknown): W, NW, SW, and at a corner those from beyond its row
    gather(a, nx - 2, y, node_flags(a.g, nx - 2, y), g);
    if (a.p.outlet_mode == kOutletCopyUnknown) {
      float own[9];
      pull(a, x, y, fl, own);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const bool unknown = CX[k] == -1 || (corner_y && (y == 0 ? CY[k] == 1 : CY[k] == -1));
        g[k] = unknown ? g[k] : own[k];
      }
      if (!corner_y) closure_outlet(a, y, g);
    }
  } else {
    gather(a, x, y, fl, g);
  }
  if (open_x && x == 0) inlet_bc(a.p, corner_y, g);
  if ((fl >> 1) && owner) {
    float own[9];
    if (a.p.interp_bb || a.p.full_bb) {
#pragma unroll
      for (int k = 0; k < 9; ++k) own[k] = load(a.A, a.g, k, x, y);
    }
    link_force(a.partial, link_slot(a.g, x, y), fl, g, own, a.p);
  }
  collide_t<COLL>(g, a.p, out, bad);
}

template <bool NT>
__device__ __forceinline__ void general_node(const StepArgs& a, int x, int y, bool& bad) {
  float out[9];
  general_update(a, x, y, true, out, bad);
  store9<NT>(a.B, (uint32_t)a.g.plane, (uint32_t)y * (uint32_t)a.g.pitch + (uint32_t)x, out);
}

__device__ __forceinline__ void bulk_update(const StepArgs& a, int x, int y, float (&out)[9], bool& bad) {
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
  collide(g, a.p, out, bad);
}

template <bool NT>
__device__ __forceinline__ void bulk_node(const StepArgs& a, int x, int y, bool& bad) {
  float out[9];
  bulk_update(a, x, y, out, bad);
  store9<NT>(a.B, (uint32_t)a.g.plane, (uint32_t)y * (uint32_t)a.g.pitch + (uint32_t)x, out);
}

template <int VX>
struct Vec;
template <>
struct Vec<2> {
  typedef float type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec<4> {
  typedef float type __attribute__((ext_vector_type(4)));
};

// VX consecutive interior nodes x0 .. x0+VX-1 of one row per lane, with every
// lane of the wave on the bulk path.  Each population plane is read with one
// aligned VX-wide load per lane; the one value a lane needs from outside its
// own span (x0-1 for the eastward-moving E, NE, SE, x0+VX for the westward
// W, NW, SW) comes from the neighbouring lane by a cross-lane shuffle, and
// only lanes 0 and 63 read it from memory.
template <int VX, bool NT>
__device__ __forceinline__ void bulk_vec(const StepArgs& a, int x0, int y, bool& bad) {
  typedef typename Vec<VX>::type V;
  const float* __restrict__ A = a.A;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
  const uint32_t o = (uint32_t)y * Wp + (uint32_t)x0;
  const uint32_t on = o - Wp, os = o + Wp;  // rows y-1 and y+1
  const V r = *(const V*)(A + o);
  const V n = *(const V*)(A + 2 * P + on);
  const V s = *(const V*)(A + 4 * P + os);
  const V e = *(const V*)(A + 1 * P + o);
  const V ne = *(const V*)(A + 5 * P + on);
  const V se = *(const V*)(A + 8 * P + os);
  const V w = *(const V*)(A + 3 * P + o);
  const V nw = *(const V*)(A + 6 * P + on);
  const V sw = *(const V*)(A + 7 * P + os);
  const int lane = (int)(threadIdx.x & 63);
  float e_in = __shfl_up(e[VX - 1], 1), ne_in = __shfl_up(ne[VX - 1], 1), se_in = __shfl_up(se[VX - 1], 1);
  float w_in = __shfl_down(w[0], 1), nw_in = __shfl_down(nw[0], 1), sw_in = __shfl_down(sw[0], 1);
  if (lane == 0) {
    e_in = A[1 * P + o - 1];
    ne_in = A[5 * P + on - 1];
    se_in = A[8 * P + os - 1];
  }
  if (lane == 63) {
    w_in = A[3 * P + o + VX];
    nw_in = A[6 * P + on + VX];
    sw_in = A[7 * P + os + VX];
  }
  V out[9];
#pragma unroll
  for (int j = 0; j < VX; ++j) {
    float g[9], f[9];
    g[0] = r[j];
    g[2] = n[j];
    g[4] = s[j];
    g[1] = j == 0 ? e_in : e[j > 0 ? j - 1 : 0];
    g[5] = j == 0 ? ne_in : ne[j > 0 ? j - 1 : 0];
    g[8] = j == 0 ? se_in : se[j > 0 ? j - 1 : 0];
    g[3] = j == VX - 1 ? w_in : w[j < VX - 1 ? j + 1 : 0];
    g[6] = j == VX - 1 ? nw_in : nw[j < VX - 1 ? j + 1 : 0];
    g[7] = j == VX - 1 ? sw_in : sw[j < VX - 1 ? j + 1 : 0];
    collide(g, a.p, f, bad);
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k][j] = f[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    V* dst = (V*)(a.B + k * P + o);
    if (NT)
      __builtin_nontemporal_store(out[k], dst);
    else
      *dst = out[k];
  }
}

// ------------------------------------------------ boundary code on registers
// The boundary treatment of a node from values already in registers, shared
// by the one-step kernel's boundary waves and every level of the multi-step
// kernels' boundary waves.

// Value of the lane below (lane l gets lane l-1) and above (lane l gets
// l+1), by DPP whole-wave shifts (a VALU move, no LDS permute).  The lane at
// the wave's end keeps its own value; only halo lanes read it.
__device__ __forceinline__ float from_left(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float from_right(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x130, 0xf, 0xf, false));
}

// What the first level of a boundary wave reads from memory for node (x, y):
// the pulled populations f*_k(x - c_k) before any boundary treatment (with
// the periodic wrap-arounds; a source outside the lattice reads the node
// itself, discarded later), the node's own f*_k for k = 1..8 (own[k - 1];
// f*_0 is pl[0]) and its raw flag and link-list entries (meaningful inside
// the cylinder rectangle only).  Every address is valid for every lane and
// nothing loaded is used here, so a wave issues the loads of the next row
// before it works on the current one and waits for them only at the end of
// that work.
struct RowIn {
  float pl[9], own[8];
  int fl, li;
};

__device__ __forceinline__ void row_load(const StepArgs& a, int x, int y, RowIn& r) {
  const int nx = a.g.nx, ny = a.g.ny;
  const int cx = min(max(x, 0), nx - 1), cy = min(max(y, 0), ny - 1);
  const float* __restrict__ A = a.A;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    int sx = x - CX[k], sy = y - CY[k];
    if (a.p.x_periodic) sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
    if (a.p.wall == kWallPeriodic) sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
    const bool ok = sx >= 0 && sx < nx && sy >= 0 && sy < ny;
    r.pl[k] = A[(uint32_t)k * P + (uint32_t)(ok ? sy : cy) * Wp + (uint32_t)(ok ? sx : cx)];
    if (k > 0) r.own[k - 1] = A[(uint32_t)k * P + (uint32_t)cy * Wp + (uint32_t)cx];
  }
  r.fl = 0;
  r.li = -1;
  if (a.g.flags) {  // a cylinder: both tables exist
    const int i = min(max(y - a.g.ry0, 0), a.g.rh - 1) * a.g.rw + min(max(x - a.g.rx0, 0), a.g.rw - 1);
    r.fl = a.g.flags[i];
    r.li = a.g.link_index[i];
  }
}

// Post-collision populations of node (x, y) one level up, from registers:
// c[k] = f*_k(x - c_k) of the level below before any boundary treatment, w1
// the node's own populations on that level, w0 and w2 those of the rows below
// and above (x-neighbours in the adjacent lanes; read for the interpolated
// bounce-back on levels above the first, L1 false), fl_raw and li the
// node's raw flag and link-list entries, rt and rb this lane's wall-row
// closure residuals.  The same steps as general_update; link forces go to
// `partial`.  On the first level (L1) the interpolated bounce-back reads
// f*_opp(k)(x + c_k) from memory (lanes at the wave's edges have no
// neighbour lane) and lanes outside the lattice get zeros; on the others
// those lanes leave `out` unset (nothing reads it).
template <int COLL, bool L1>
__device__ __forceinline__ void update_regs(const StepArgs& a, double2* __restrict__ partial, int x, int y,
                                            bool active, bool owner, const float (&c)[9], const float (&w0)[9],
                                            const float (&w1)[9], const float (&w2)[9], int fl_raw, int li,
                                            const float (&rt)[3], const float (&rb)[3], float (&out)[9],
                                            bool& bad) {
  const int nx = a.g.nx, ny = a.g.ny;
  const bool inr = in_rect(a.g, x, y);
  const bool special = active && (x == 0 || x >= nx - 1 || y == 0 || y == ny - 1 || inr);
  bool b = false;
  if (!__any(special)) {
    if (active) collide_t<COLL>(c, a.p, out, b);
  } else {
    const bool open_x = !a.p.x_periodic;
    const bool outlet = active && open_x && x == nx - 1;
    const bool corner_y = a.p.wall != kWallPeriodic && (y == 0 || y == ny - 1);
    const uint16_t fl = active && inr ? (uint16_t)fl_raw : 0;
    // interpolated bounce-back needs f*_opp(k) at x + c_k (only where the
    // wave has links)
    float bh[9];
    const bool interp = a.p.interp_bb && __any(fl >> 1);
    if (interp) {
      if (L1) {
        bh[0] = 0.0f;
#pragma unroll
        for (int k = 1; k < 9; ++k)  // the cylinder keeps two nodes from every edge: x + c_k is inside
          bh[k] = ((fl >> k) & 1) ? load(a.A, a.g, OPP[k], x + CX[k], y + CY[k]) : 0.0f;
      } else {
        bh[0] = 0.0f;
        bh[1] = from_right(w1[3]);
        bh[2] = w2[4];
        bh[3] = from_left(w1[1]);
        bh[4] = w0[2];
        bh[5] = from_right(w2[7]);
        bh[6] = from_left(w2[8]);
        bh[7] = from_left(w0[5]);
        bh[8] = from_right(w0[6]);
      }
    }
    // Streamed values; a source outside the lattice exists only across an
    // open edge (with the periodic modes the lanes and rows already hold the
    // wrapped neighbours), and its population is one of the missing ones,
    // set to zero for the corrections below.  Every test that picks the work
    // is uniform across the wave: the row is the same for all lanes.
    float g[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) g[k] = c[k];
    if (open_x && __any(active && (x == 0 || x == nx - 1))) {
      const bool w = x == 0, e = x == nx - 1;
      g[1] = w ? 0.0f : g[1];
      g[5] = w ? 0.0f : g[5];
      g[8] = w ? 0.0f : g[8];
      g[3] = e ? 0.0f : g[3];
      g[6] = e ? 0.0f : g[6];
      g[7] = e ? 0.0f : g[7];
    }
    const bool wall_row = a.p.wall != kWallPeriodic && (y == 0 || y == ny - 1);
    if (wall_row) {
      const bool s0 = y == 0;
      g[2] = s0 ? 0.0f : g[2];
      g[5] = s0 ? 0.0f : g[5];
      g[6] = s0 ? 0.0f : g[6];
      g[4] = s0 ? g[4] : 0.0f;
      g[7] = s0 ? g[7] : 0.0f;
      g[8] = s0 ? g[8] : 0.0f;
    }
    if (!a.p.full_bb && __any(fl >> 1)) {  // bounce-back on the cylinder
#pragma unroll
      for (int k = 1; k < 9; ++k) {
        if (!((fl >> k) & 1)) continue;
        if (interp) {
          const float q = a.g.q[8 * li + k - 1];
          g[k] = bfl(q, w1[OPP[k]], bh[k], w1[k]);
        } else {
          g[k] = w1[OPP[k]];
        }
      }
    }
    const bool wall_x = a.p.x_periodic || (x >= 1 && x <= nx - 2);
    if (active && wall_row && wall_x) {
      wall_bc(a.p, y == ny - 1, w1, g);
      closure_row_regs(a, y == ny - 1, rt, rb, g);
    }
    // Eq. 13: the corrected populations of x = nx-2 are the left lane's g
    if (__any(outlet)) {
      float G[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) G[k] = from_left(g[k]);
      if (outlet) {
        if (a.p.outlet_mode == kOutletCopyUnknown) {
          // only what streams in from outside: W, NW, SW, and at a corner
          // the populations from beyond its row
#pragma unroll
          for (int k = 0; k < 9; ++k) {
            const bool unknown = CX[k] == -1 || (corner_y && (y == 0 ? CY[k] == 1 : CY[k] == -1));
            g[k] = unknown ? G[k] : g[k];
          }
          if (!corner_y) closure_outlet(a, y, g);
        } else {
#pragma unroll
          for (int k = 0; k < 9; ++k) g[k] = G[k];
        }
      }
    }
    if (active) {
      if (fl & kSolid) {
#pragma unroll
        for (int k = 0; k < 9; ++k) out[k] = a.p.full_bb ? g[OPP[k]] : w1[k];
      } else {
        if (open_x && x == 0) inlet_bc(a.p, corner_y, g);
        if ((fl >> 1) && owner) link_force(partial, li, fl, g, w1, a.p);
        collide_t<COLL>(g, a.p, out, b);
      }
    }
  }
  if (L1 && !active) {
#pragma unroll
    for (int k = 0; k < 9; ++k) out[k] = 0.0f;
  }
  bad |= b && owner;
}

// Records a failed density check of step `slot` once per wave (one atomic
// per wave rather than per node keeps a diverged lattice, where every node
// fails, from serialising on the flag).  Every lane of the wave must call it.
__device__ __forceinline__ void report_bad(int* flag, bool bad, int slot) {
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicMin(flag, slot);
}

// Blocks are dispatched round-robin over the 8 XCDs (block id mod 8), and
// each XCD has its own L2.  Two block-to-tile maps keep neighbouring tiles of
// a row, which share the halo cache lines of the x-shifted planes, on one XCD:
//  1: each XCD gets a contiguous range of tiles (a band of rows);
//  2: XCD i gets the tile rows congruent to i mod 8, in row order, so all
//     eight still sweep the lattice together (one narrow band of rows at any
//     time, as with the plain order) and a row's tiles meet in one L2.
// Tile rows past the last complete group of eight keep the plain order.
__device__ __forceinline__ int remap_xcd(int id, int n) {
  const int xcd = id & 7, local = id >> 3;
  const int per = n >> 3, rem = n & 7;
  return xcd * per + min(xcd, rem) + local;
}

__device__ __forceinline__ int remap_xcd_rows(int id, int ntx, int nty) {
  const int full = (nty >> 3) * ntx * 8;
  if (id >= full) return id;
  const int xcd = id & 7, local = id >> 3;
  const int r = local / ntx, t = local - r * ntx;
  return (8 * r + xcd) * ntx + t;
}

// One tile = tile_x = 256 * VX consecutive nodes of TY rows; lane t of the
// block owns nodes x0 .. x0+VX-1 with x0 = tile origin + VX t.  Waves with a
// node that needs the boundary code load everything it may read at once and
// apply it on registers (update_regs) when each lane holds one node and the
// outlet's left neighbour is in the same wave; otherwise node by node
// (general_node).
template <int TY, int VX, bool NT>
__device__ __forceinline__ void process_tile(const StepArgs& a, int bx, int by) {
  const int nx = a.g.nx, ny = a.g.ny;
  const int x0 = bx * a.t.tile_x + (int)threadIdx.x * VX;
  bool bad = false;
#pragma unroll
  for (int r = 0; r < TY; ++r) {
    const int y = by * TY + r;
    const bool active = x0 < nx && y < ny;
    const bool rect = (unsigned)(y - a.g.ry0) < (unsigned)a.g.rh && x0 + VX - 1 >= a.g.rx0 &&
                      x0 < a.g.rx0 + a.g.rw;
    const bool special = active && (x0 == 0 || x0 + VX - 1 >= nx - 1 || y == 0 || y == ny - 1 || rect);
    if (__any(special)) {
      if (VX == 1 && (a.p.x_periodic || ((nx - 1) & 63) != 0)) {
        RowIn in;
        row_load(a, x0, y, in);
        float rt[3], rb[3];
        closure_rows_load(a, y == 0 || y == ny - 1, x0, rt, rb);
        float own[9], out[9];
        own[0] = in.pl[0];
#pragma unroll
        for (int k = 1; k < 9; ++k) own[k] = in.own[k - 1];
        update_regs<kEither, true>(a, a.partial, x0, y, active, true, in.pl, own, own, own, in.fl, in.li, rt, rb,
                                   out, bad);
        if (active) store9<NT>(a.B, (uint32_t)a.g.plane, (uint32_t)y * (uint32_t)a.g.pitch + (uint32_t)x0, out);
      } else {
#pragma unroll
        for (int j = 0; j < VX; ++j)
          if (active && x0 + j < nx) general_node<NT>(a, x0 + j, y, bad);
      }
    } else if (active) {
      if constexpr (VX == 1)
        bulk_node<NT>(a, x0, y, bad);
      else
        bulk_vec<VX, NT>(a, x0, y, bad);
    }
  }
  report_bad(a.bad, bad, a.slot);
}

template <int TY, int VX, bool NT>
__global__ __launch_bounds__(256) void step_kernel(StepArgs a) {
  const int ntiles = a.t.ntx * a.t.nty;
  const int id = (int)blockIdx.x;
  const int tile = a.t.remap_xcd == 1   ? remap_xcd(id, ntiles)
                   : a.t.remap_xcd == 2 ? remap_xcd_rows(id, a.t.ntx, a.t.nty)
                                        : id;
  process_tile<TY, VX, NT>(a, tile % a.t.ntx, tile / a.t.ntx);
}

// ---------------------------------------------------------------------------
// Two time steps per launch, the intermediate state kept in registers.
//
// Each wave owns a strip of kStrip2 = 62 output columns and a segment of
// tile_y output rows; its 64 lanes hold the columns from one left of the strip
// to one right of it.  The wave walks its segment down in y.  At row r it
// computes f*(t+1) from memory for all 64 lanes and keeps it; the rows r-2,
// r-1 and r of f*(t+1) then give f*(t+2) at row r-1, pulled from registers
// (the x-neighbours by cross-lane moves), and only that is written.  One
// launch thus reads and writes each population once for two node updates.
// The edge lanes and the rows just outside the segment are computed by two
// waves, but each node's output, force contribution and density check come
// from its owner only.  Every node sees the same FP32 values and the same
// arithmetic as in two one-step launches, so the results are equal bit for
// bit.
//
// Segments whose first-step nodes are all plain bulk fluid (interior_segment)
// run a lean, fully unrolled path (bulk_wave); the others run the boundary
// code of the one-step kernel on registers (general_wave_n, update_regs).
// Without x-periodicity the strips are aligned to the right
// edge, so the outlet column is always lane 62 and the column it copies
// (nx-2) lane 61.
// The nine pulled values of bulk node (x, y).
__device__ __forceinline__ void load_pull(const StepArgs& a, int x, int y, float (&v)[9]) {
  const float* __restrict__ A = a.A;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
  const uint32_t o = (uint32_t)y * Wp + (uint32_t)x;
  v[0] = A[o];
  v[1] = A[P + o - 1];
  v[2] = A[2 * P + o - Wp];
  v[3] = A[3 * P + o + 1];
  v[4] = A[4 * P + o + Wp];
  v[5] = A[5 * P + o - Wp - 1];
  v[6] = A[6 * P + o - Wp + 1];
  v[7] = A[7 * P + o + Wp + 1];
  v[8] = A[8 * P + o + Wp - 1];
}

// Interior waves, H = tile_y rows.  The row loop is unrolled; its loads run
// two rows ahead (every load first for H <= 6), and the H output rows stay
// in registers until every load of the wave has been issued, so no load
// waits behind a store (on this chip one counter tracks both, and a wait for
// a load also waits for the older stores).
template <bool NT, int H>
__device__ __forceinline__ void bulk_wave(const StepArgs& a, int strip, int seg) {
  const int lane = (int)(threadIdx.x & 63);
  if (!interior_segment(a.g, a.t, a.p.x_periodic, strip, seg)) return;
  const int xs = strip_start(a.g, a.t, a.p.x_periodic, strip);
  const int y0 = seg * H;
  const int x = xs - 1 + lane;
  const bool out_col = lane >= 1 && lane <= kStrip2;
  constexpr int AHEAD = H <= 6 ? H + 2 : 2, R = AHEAD + 1;
  float w[3][9], pre[R][9], out[H][9];
#pragma unroll
  for (int i = 0; i < AHEAD; ++i) load_pull(a, x, y0 - 1 + i, pre[i]);
  bool bad1 = false, bad2 = false;
#pragma unroll
  for (int i = 0; i < H + 2; ++i) {  // f*(t+1) of row y0-1+i
    if (i + AHEAD < H + 2) load_pull(a, x, y0 - 1 + i + AHEAD, pre[(i + AHEAD) % R]);
    bool b1 = false;
    collide(pre[i % R], a.p, w[i % 3], b1);
    if (i >= 1 && i <= H) bad1 |= b1;
    if (i >= 2) {  // f*(t+2) of row y0+i-2
      const float(&wa)[9] = w[(i + 1) % 3];
      const float(&wb)[9] = w[(i + 2) % 3];
      const float(&wc)[9] = w[i % 3];
      float c[9];
      c[0] = wb[0];
      c[1] = from_left(wb[1]);
      c[2] = wa[2];
      c[3] = from_right(wb[3]);
      c[4] = wc[4];
      c[5] = from_left(wa[5]);
      c[6] = from_right(wa[6]);
      c[7] = from_right(wc[7]);
      c[8] = from_left(wc[8]);
      collide(c, a.p, out[i - 2], bad2);
    }
  }
  report_bad(a.bad, bad1 && out_col, a.slot);
  report_bad(a.bad, bad2 && out_col, a.slot + 1);
  if (!out_col) return;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
#pragma unroll
  for (int j = 0; j < H; ++j) store9<NT>(a.B, P, (uint32_t)(y0 + j) * Wp + (uint32_t)x, out[j]);
}

// ------------------------------------------------------- three or four steps
// The same scheme S - 1 levels deeper (S = 3 or 4 steps per launch): each
// wave's 64 lanes hold its 64 - 2(S-1) output columns (kStrip3 = 60,
// kStrip4 = 58) and S - 1 more on either side; f*(t+1) is computed from
// memory on the segment's rows widened by S - 1 on each side, each further
// level from the one below it in registers on rows widened by one less, and
// only f*(t+S) is stored.

// Pulled values of a node from the level below, held as rows above (wa), at
// (wb) and below (wc) the node, x-neighbours in the adjacent lanes.
__device__ __forceinline__ void pull_rows(const float (&wa)[9], const float (&wb)[9], const float (&wc)[9],
                                          float (&c)[9]) {
  c[0] = wb[0];
  c[1] = from_left(wb[1]);
  c[2] = wa[2];
  c[3] = from_right(wb[3]);
  c[4] = wc[4];
  c[5] = from_left(wa[5]);
  c[6] = from_right(wa[6]);
  c[7] = from_right(wc[7]);
  c[8] = from_left(wc[8]);
}

// Force contributions of level l (1-based) of a multi-step launch.
__device__ __forceinline__ double2* level_partial(const StepArgs& a, int l) {
  return l == 1 ? a.partial : l == 2 ? a.partial2 : l == 3 ? a.partial3 : a.partial4;
}

// Interior segments, H rows.  Iteration i computes level 1 on row
// y0 - h + i from memory and level l on row y0 - h + i - (l - 1) from the
// rows of level l - 1 made in iterations i - 2 .. i; loads run AHEAD rows
// ahead of level 1 (all of them first when they fit), outputs are stored at
// the end.  The collision operator is fixed at compile time (COLL): the
// kernel's code then holds one operator's bulk path only, which keeps it
// within the instruction cache better.
template <bool NT, int H, int S, int COLL>
__device__ __forceinline__ void bulk_wave_n(const StepArgs& a, int strip, int seg) {
  constexpr int h = S - 1, W = 64 - 2 * h;
  const int lane = (int)(threadIdx.x & 63);
  if (!interior_segment(a.g, a.t, a.p.x_periodic, strip, seg)) return;
  const int xs = strip_start(a.g, a.t, a.p.x_periodic, strip);
  const int y0 = seg * H;
  const int x = xs - h + lane;
  const bool out_col = lane >= h && lane < h + W;
  constexpr int N1 = H + 2 * h;  // first-level rows y0-h .. y0+H+h-1
  constexpr int AHEAD = N1 <= 8 ? N1 : 3, R = AHEAD + 1;
  float w[S - 1][3][9], pre[R][9], out[H][9];
#pragma unroll
  for (int i = 0; i < AHEAD; ++i) load_pull(a, x, y0 - h + i, pre[i]);
  bool bad[S];
#pragma unroll
  for (int l = 0; l < S; ++l) bad[l] = false;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    if (i + AHEAD < N1) load_pull(a, x, y0 - h + i + AHEAD, pre[(i + AHEAD) % R]);
    bool b1 = false;
    collide_t<COLL>(pre[i % R], a.p, w[0][i % 3], b1);
    if (i >= h && i < h + H) bad[0] |= b1;
#pragma unroll
    for (int l = 2; l <= S; ++l) {
      if (i < 2 * (l - 1)) continue;
      float c[9];
      pull_rows(w[l - 2][(i + 1) % 3], w[l - 2][(i + 2) % 3], w[l - 2][i % 3], c);
      if (l < S) {
        bool b = false;
        collide_t<COLL>(c, a.p, w[l - 1][i % 3], b);
        const int q = i - h - (l - 1);  // row - y0
        if (q >= 0 && q < H) bad[l - 1] |= b;
      } else {
        collide_t<COLL>(c, a.p, out[i - 2 * h], bad[S - 1]);
      }
    }
  }
#pragma unroll
  for (int l = 0; l < S; ++l) report_bad(a.bad, bad[l] && out_col, a.slot + l);
  if (!out_col) return;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
#pragma unroll
  for (int j = 0; j < H; ++j) store9<NT>(a.B, P, (uint32_t)(y0 + j) * Wp + (uint32_t)x, out[j]);
}

// Interior segments with each output row stored as soon as it is made
// (variants "tS_hHu_*").  bulk_wave_n holds the H output rows of a segment
// in registers and stores them at the end, which keeps loads from waiting
// behind stores but bounds H (8 rows: 72 registers of outputs), and short
// segments recompute and re-read their 2(S - 1) halo rows per level for few
// output rows (14 first-level rows for 8 at S = 4).  Here the registers hold
// only the three newest rows of each level below the last and the loads in
// flight, whatever H: at H = 16, 22 + 20 + 18 + 16 rows are updated for
// 16 x 4 output rows (1.19 times the useful updates against 1.38 at H = 8)
// and 24 rows of each plane are read for 16 (1.5 against 2).  The row loop
// is unrolled, like bulk_wave_n's, so every ring index and every test on the
// row is a constant and the compiler's waits on the loads are exact: rolled
// over groups of rows (with the rows' tests at run time), the compiler
// waited for every load in flight once per group and the tall segments ran
// slower than the short ones despite their smaller traffic.  Stores now sit
// between loads; the wait for a row's loads also waits for the stores issued
// before them, which left AHEAD iterations earlier.
template <bool NT, int H, int S, int COLL, int AHEAD>
__device__ __forceinline__ void bulk_wave_s(const StepArgs& a, int strip, int seg) {
  constexpr int h = S - 1, W = 64 - 2 * h;
  constexpr int R = AHEAD + 1;
  constexpr int N1 = H + 2 * h;  // first-level rows y0-h .. y0+H+h-1
  const int lane = (int)(threadIdx.x & 63);
  if (!interior_segment(a.g, a.t, a.p.x_periodic, strip, seg)) return;
  const int xs = strip_start(a.g, a.t, a.p.x_periodic, strip);
  const int y0 = seg * H;
  const int x = xs - h + lane;
  const bool out_col = lane >= h && lane < h + W;
  const uint32_t Pl = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
  float w[S - 1][3][9], pre[R][9];
#pragma unroll
  for (int i = 0; i < AHEAD; ++i) load_pull(a, x, y0 - h + i, pre[i]);
  bool bad[S];
#pragma unroll
  for (int l = 0; l < S; ++l) bad[l] = false;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    if (i + AHEAD < N1) load_pull(a, x, y0 - h + i + AHEAD, pre[(i + AHEAD) % R]);
    bool b1 = false;
    collide_t<COLL>(pre[i % R], a.p, w[0][i % 3], b1);
    if (i >= h && i < h + H) bad[0] |= b1;
#pragma unroll
    for (int l = 2; l <= S; ++l) {
      if (i < 2 * (l - 1)) continue;
      float c[9];
      pull_rows(w[l - 2][(i + 1) % 3], w[l - 2][(i + 2) % 3], w[l - 2][i % 3], c);
      const int q = i - h - (l - 1);  // row - y0 of this level's row
      if (l < S) {
        bool b = false;
        collide_t<COLL>(c, a.p, w[l - 1][i % 3], b);
        if (q >= 0 && q < H) bad[l - 1] |= b;
      } else {
        float out[9];
        collide_t<COLL>(c, a.p, out, bad[S - 1]);
        if (out_col) store9<NT>(a.B, Pl, (uint32_t)(y0 + q) * Wp + (uint32_t)x, out);
      }
    }
  }
#pragma unroll
  for (int l = 0; l < S; ++l) report_bad(a.bad, bad[l] && out_col, a.slot + l);
}

// SUB rows (fewer at the segment's or the lattice's end) of a segment that
// is not interior, with the boundary code on every level: a rolled loop over
// the first-level rows r, each level l > 1 following on row r - (l - 1).
// Each pass issues the loads of row r + 1 first and waits for them only when
// it moves them into place at its end, so the boundary code of the S levels
// runs while they are in flight; nothing else in the loop reads memory
// (except the interpolated bounce-back's wall fractions and the outlet
// closure's residuals).  Rolled, because unrolled copies of the boundary
// code crowd the instruction cache that the bulk waves on the same CU run
// from.
template <bool NT, int SUB, int S, int COLL>
__device__ __forceinline__ void general_wave_n(const StepArgs& a, int segment, int sub) {
  constexpr int h = S - 1, W = 64 - 2 * h;
  const int lane = (int)(threadIdx.x & 63);
  const int St = a.t.ntx, H = a.t.tile_y;
  const int strip = segment % St, seg = segment / St;
  const int nx = a.g.nx, ny = a.g.ny;
  const bool xper = a.p.x_periodic, yper = a.p.wall == kWallPeriodic;
  const int xs = strip_start(a.g, a.t, xper, strip);
  const int y0 = seg * H + sub * SUB;
  if (y0 >= ny) return;
  const int y1 = min(min(y0 + SUB, seg * H + H), ny);
  const int ux = xs - h + lane;  // column before wrapping
  const int x = xper ? ((ux % nx) + nx) % nx : ux;
  const bool col_ok = xper || (ux >= 0 && ux < nx);
  const bool out_col = lane >= h && lane < h + W && ux >= 0 && ux < nx;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
  auto row_of = [&](int r) { return yper ? (r < 0 ? r + ny : (r >= ny ? r - ny : r)) : r; };
  auto row_ok = [&](int r) { return yper || (r >= 0 && r < ny); };
  float rt[3], rb[3];
  closure_rows_load(a, y0 - h <= 0 || y1 + h - 1 >= ny - 1, x, rt, rb);
  float lv[S - 1][3][9];  // rows q-1, q, q+1 of each level below the last
#pragma unroll
  for (int l = 0; l < S - 1; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 9; ++k) lv[l][j][k] = 0.0f;
  int fr[S], lr[S];  // raw flag and link entries of rows r, r-1, ..., r-S+1
#pragma unroll
  for (int j = 0; j < S; ++j) {
    fr[j] = 0;
    lr[j] = -1;
  }
  RowIn cur, nxt;
  row_load(a, x, row_of(y0 - h), cur);
  bool bad[S];
#pragma unroll
  for (int l = 0; l < S; ++l) bad[l] = false;
#pragma unroll 1
  for (int r = y0 - h; r <= y1 + h - 1; ++r) {
    row_load(a, x, row_of(r + 1), nxt);
#pragma unroll
    for (int j = S - 1; j > 0; --j) {
      fr[j] = fr[j - 1];
      lr[j] = lr[j - 1];
    }
    fr[0] = cur.fl;
    lr[0] = cur.li;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      lv[0][0][k] = lv[0][1][k];
      lv[0][1][k] = lv[0][2][k];
    }
    {  // level 1 (f*(t+1)) of row r
      float own[9];
      own[0] = cur.pl[0];
#pragma unroll
      for (int k = 1; k < 9; ++k) own[k] = cur.own[k - 1];
      update_regs<COLL, true>(a, a.partial, x, row_of(r), col_ok && row_ok(r), out_col && r >= y0 && r < y1,
                              cur.pl, own, own, own, fr[0], lr[0], rt, rb, lv[0][2], bad[0]);
    }
#pragma unroll
    for (int l = 2; l <= S; ++l) {
      if (r < y0 - h + 2 * (l - 1)) continue;
      const int q = r - (l - 1);  // level l of row q
      float c[9];
      pull_rows(lv[l - 2][0], lv[l - 2][1], lv[l - 2][2], c);
      if (l < S) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          lv[l - 1][0][k] = lv[l - 1][1][k];
          lv[l - 1][1][k] = lv[l - 1][2][k];
        }
        update_regs<COLL, false>(a, level_partial(a, l), x, row_of(q), col_ok && row_ok(q),
                                 out_col && q >= y0 && q < y1, c, lv[l - 2][0], lv[l - 2][1], lv[l - 2][2],
                                 fr[l - 1], lr[l - 1], rt, rb, lv[l - 1][2], bad[l - 1]);
      } else {
        float out[9];
        update_regs<COLL, false>(a, level_partial(a, l), x, q, col_ok, out_col, c, lv[l - 2][0], lv[l - 2][1],
                                 lv[l - 2][2], fr[l - 1], lr[l - 1], rt, rb, out, bad[S - 1]);
        if (out_col) store9<NT>(a.B, P, (uint32_t)q * Wp + (uint32_t)x, out);
      }
    }
    cur = nxt;
  }
#pragma unroll
  for (int l = 0; l < S; ++l) report_bad(a.bad, bad[l], a.slot + l);
}

// A boundary piece as in general_wave_n, with the loads of all its
// SUB + 2(S - 1) first-level rows issued before any update and no row loop:
// the piece's serial chain is one memory latency plus its updates, the
// first-level rows independent of each other, which suits short launches
// (lattices of a few hundred thousand nodes) at the cost of more registers
// and code.  Rows past the end of a short piece are loaded (clamped) but
// not worked on, as in the loop.
template <bool NT, int SUB, int S, int COLL>
__device__ __forceinline__ void general_wave_u(const StepArgs& a, int segment, int sub) {
  constexpr int h = S - 1, W = 64 - 2 * h, N1 = SUB + 2 * h;
  const int lane = (int)(threadIdx.x & 63);
  const int St = a.t.ntx, H = a.t.tile_y;
  const int strip = segment % St, seg = segment / St;
  const int nx = a.g.nx, ny = a.g.ny;
  const bool xper = a.p.x_periodic, yper = a.p.wall == kWallPeriodic;
  const int xs = strip_start(a.g, a.t, xper, strip);
  const int y0 = seg * H + sub * SUB;
  if (y0 >= ny) return;
  const int y1 = min(min(y0 + SUB, seg * H + H), ny);
  const int ux = xs - h + lane;  // column before wrapping
  const int x = xper ? ((ux % nx) + nx) % nx : ux;
  const bool col_ok = xper || (ux >= 0 && ux < nx);
  const bool out_col = lane >= h && lane < h + W && ux >= 0 && ux < nx;
  const uint32_t P = (uint32_t)a.g.plane, Wp = (uint32_t)a.g.pitch;
  auto row_of = [&](int r) { return yper ? (r < 0 ? r + ny : (r >= ny ? r - ny : r)) : r; };
  auto row_ok = [&](int r) { return yper || (r >= 0 && r < ny); };
  RowIn in[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) row_load(a, x, row_of(y0 - h + i), in[i]);
  float rt[3], rb[3];
  closure_rows_load(a, y0 - h <= 0 || y1 + h - 1 >= ny - 1, x, rt, rb);
  float lv[S - 1][3][9];
#pragma unroll
  for (int l = 0; l < S - 1; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
      for (int k = 0; k < 9; ++k) lv[l][j][k] = 0.0f;
  bool bad[S];
#pragma unroll
  for (int l = 0; l < S; ++l) bad[l] = false;
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    const int r = y0 - h + i;
    if (r > y1 + h - 1) break;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      lv[0][0][k] = lv[0][1][k];
      lv[0][1][k] = lv[0][2][k];
    }
    {  // level 1 (f*(t+1)) of row r
      float own[9];
      own[0] = in[i].pl[0];
#pragma unroll
      for (int k = 1; k < 9; ++k) own[k] = in[i].own[k - 1];
      update_regs<COLL, true>(a, a.partial, x, row_of(r), col_ok && row_ok(r), out_col && r >= y0 && r < y1,
                              in[i].pl, own, own, own, in[i].fl, in[i].li, rt, rb, lv[0][2], bad[0]);
    }
#pragma unroll
    for (int l = 2; l <= S; ++l) {
      if (i < 2 * (l - 1)) continue;
      const int q = r - (l - 1);  // level l of row q
      const RowIn& iq = in[i - (l - 1)];
      float c[9];
      pull_rows(lv[l - 2][0], lv[l - 2][1], lv[l - 2][2], c);
      if (l < S) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          lv[l - 1][0][k] = lv[l - 1][1][k];
          lv[l - 1][1][k] = lv[l - 1][2][k];
        }
        update_regs<COLL, false>(a, level_partial(a, l), x, row_of(q), col_ok && row_ok(q),
                                 out_col && q >= y0 && q < y1, c, lv[l - 2][0], lv[l - 2][1], lv[l - 2][2], iq.fl,
                                 iq.li, rt, rb, lv[l - 1][2], bad[l - 1]);
      } else {
        float out[9];
        update_regs<COLL, false>(a, level_partial(a, l), x, q, col_ok, out_col, c, lv[l - 2][0], lv[l - 2][1],
                                 lv[l - 2][2], iq.fl, iq.li, rt, rb, out, bad[S - 1]);
        if (out_col) store9<NT>(a.B, P, (uint32_t)q * Wp + (uint32_t)x, out);
      }
    }
  }
#pragma unroll
  for (int l = 0; l < S; ++l) report_bad(a.bad, bad[l], a.slot + l);
}

// One launch, two steps.  The first blocks take the boundary sub-segments
// (segments listed on the host, cut into SUB rows each so that they run
// alongside the interior ones: 2 rows keep them short where the launch is
// short, 4 halve their recomputed rows where it is long); the later blocks
// one segment per wave, in
// row-major order of (segment, strip), so that the waves in flight at any
// time cover a narrow band of rows, four neighbouring strips per block.
// (Orders that keep vertically adjacent segments on one XCD, so that their
// shared rows are read once into its L2, fetch 30 % fewer bytes but ran
// 4-10 % slower: the plain order's DRAM locality wins.)
// With CLO the launch's first a.ev.blocks blocks evaluate the learned
// closure's network on the state the launch starts from (closure_block, in
// the dynamic LDS), alongside the steps, which apply the residuals of the
// previous evaluation: the evaluation then costs no launch of its own.  The
// launches without an evaluation run the instance without that code (its
// mere presence cost 2-4 % on the 458 k-node closure window).
template <bool NT, int H, int SUB, bool UNR, bool CLO>
__global__ __launch_bounds__(256) void step2_kernel(StepArgs a) {
  int b = (int)blockIdx.x;
  if constexpr (CLO) {
    if (b < a.ev.blocks) {
      extern __shared__ __align__(16) unsigned char dyn[];
      closure_block(a.ev, a.A, a.g, b, *reinterpret_cast<FwdLds*>(dyn),
                    reinterpret_cast<uint16_t*>(dyn + sizeof(FwdLds)));
      return;
    }
    b -= a.ev.blocks;
  }
  constexpr int per = (H + SUB - 1) / SUB;
  const int gen_blocks = (a.n_gen * per + 3) / 4;
  const int w = (int)(threadIdx.x >> 6);
  if (b < gen_blocks) {
    const int wave = b * 4 + w;
    if (wave < a.n_gen * per) {
      if constexpr (UNR)
        general_wave_u<NT, SUB, 2, kEither>(a, a.gen[wave / per], wave % per);
      else
        general_wave_n<NT, SUB, 2, kEither>(a, a.gen[wave / per], wave % per);
    }
    return;
  }
  const int wave = (b - gen_blocks) * 4 + w;
  if (wave < a.t.ntx * a.t.nty) bulk_wave<NT, H>(a, wave % a.t.ntx, wave / a.t.ntx);
}

// One launch, S steps; blocks as in step2_kernel.
template <bool NT, int H, int SUB, int S, int COLL, int STREAM>
__global__ __launch_bounds__(256) void multistep_kernel(StepArgs a) {
  constexpr int per = (H + SUB - 1) / SUB;
  const int gen_blocks = (a.n_gen * per + 3) / 4;
  const int b = (int)blockIdx.x, w = (int)(threadIdx.x >> 6);
  if (b < gen_blocks) {
    const int wave = b * 4 + w;
    if (wave < a.n_gen * per) general_wave_n<NT, SUB, S, COLL>(a, a.gen[wave / per], wave % per);
    return;
  }
  const int wave = (b - gen_blocks) * 4 + w;
  if (wave >= a.t.ntx * a.t.nty) return;
  if constexpr (STREAM > 0)
    bulk_wave_s<NT, H, S, COLL, STREAM>(a, wave % a.t.ntx, wave / a.t.ntx);
  else
    bulk_wave_n<NT, H, S, COLL>(a, wave % a.t.ntx, wave / a.t.ntx);
}

// One step of a whole ensemble: block b processes tile tiles[b] = (case,
// tile index within the case) with that case's geometry, physics, buffers
// and force slots, through the same per-node code as step_kernel, so every
// case evolves bit for bit as it would alone.
template <int TY, int VX, bool NT>
__global__ __launch_bounds__(256) void step_batch_kernel(const CaseArgs* __restrict__ cases,
                                                         const int2* __restrict__ tiles, int cur,
                                                         int slot, int partial_stride) {
  const int2 ct = tiles[blockIdx.x];
  const CaseArgs& c = cases[ct.x];
  StepArgs a{};  // every field not set below (closure, second-step slots) is null
  a.A = c.buf[cur];
  a.B = c.buf[cur ^ 1];
  a.g = c.g;
  a.p = c.p;
  a.t = c.t;
  a.partial = c.partial + (size_t)slot * partial_stride;
  a.bad = c.bad;
  a.slot = slot;
  process_tile<TY, VX, NT>(a, ct.y % c.t.ntx, ct.y / c.t.ntx);
}

// S steps of a whole ensemble in one launch: wave w takes task w of the
// boundary list (w < n_gen) or task w - n_gen of the interior list, each a
// (case, code) pair: code = seg * ntx + strip of the case's multi-step
// tiling for an interior segment, (seg * ntx + strip) * pieces + piece for
// a boundary piece.  The wave then runs the single-lattice wave code
// with that case's buffers, geometry, physics and force slots, so every case
// evolves bit for bit as it would alone.  Boundary pieces come first, as in
// multistep_kernel.
template <bool NT, int H, int SUB, int S, int STREAM>
__global__ __launch_bounds__(256) void multistep_batch_kernel(const CaseArgs* __restrict__ cases,
                                                              const int2* __restrict__ gen_tasks, int n_gen,
                                                              const int2* __restrict__ bulk_tasks, int n_bulk,
                                                              int cur, int slot, int partial_stride) {
  constexpr int per = (H + SUB - 1) / SUB;
  const int wave = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (wave >= n_gen + n_bulk) return;
  const bool general = wave < n_gen;
  const int2 task = general ? gen_tasks[wave] : bulk_tasks[wave - n_gen];
  const int ci = __builtin_amdgcn_readfirstlane(task.x);
  const int code = __builtin_amdgcn_readfirstlane(task.y);
  const CaseArgs& c = cases[ci];
  StepArgs a{};  // no closure, no boundary list (the task names the segment)
  a.A = c.buf[cur];
  a.B = c.buf[cur ^ 1];
  a.g = c.g;
  a.p = c.p;
  a.t = c.tm;
  a.partial = c.partial + (size_t)slot * partial_stride;
  a.partial2 = a.partial + partial_stride;
  a.partial3 = S >= 3 ? a.partial2 + partial_stride : nullptr;
  a.partial4 = S >= 4 ? a.partial3 + partial_stride : nullptr;
  a.bad = c.bad;
  a.slot = slot;
  if (general)
    general_wave_n<NT, SUB, S, kEither>(a, code / per, code % per);
  else if constexpr (STREAM > 0)
    bulk_wave_s<NT, H, S, kEither, STREAM>(a, code % a.t.ntx, code / a.t.ntx);
  else
    bulk_wave_n<NT, H, S, kEither>(a, code % a.t.ntx, code / a.t.ntx);
}

// Folds row blockIdx.x of the per-node force contributions into the FP64
// history at step *dev_step + blockIdx.x.  The order is fixed: thread t sums
// nodes t, t+256, ... in turn, each wave reduces its 64 sums by a butterfly
// of shuffles, and thread 0 adds the four wave sums in wave order.  The grid
// holds one block per pending step; when more steps are pending than the
// history holds, only the newest `cap` of them are written (two blocks would
// otherwise share a slot in no fixed order).
__global__ __launch_bounds__(256) void force_reduce_kernel(const double2* __restrict__ partials,
                                                           int nnodes, double* hist, int64_t cap,
                                                           const int64_t* dev_step) {
  __shared__ double2 wsum[4];
  const int j = blockIdx.x;
  if ((int64_t)j + cap < (int64_t)gridDim.x) return;  // uniform per block
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < nnodes; i += 256) {
    const double2 v = partials[(int64_t)j * nnodes + i];
    sx += v.x;
    sy += v.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sx += __shfl_xor(sx, off);
    sy += __shfl_xor(sy, off);
  }
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = make_double2(sx, sy);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double fx = (wsum[0].x + wsum[1].x) + (wsum[2].x + wsum[3].x);
    const double fy = (wsum[0].y + wsum[1].y) + (wsum[2].y + wsum[3].y);
    const int64_t s = (*dev_step + j) % cap;
    hist[2 * s] = fx;
    hist[2 * s + 1] = fy;
  }
}

// Ensemble version of the two kernels below: block (j, c) folds step j of
// case c (cases [0, ncases) are the active ones) exactly as
// force_reduce_kernel folds a single lattice's step, newest hist_cap steps
// only.
__global__ __launch_bounds__(256) void force_reduce_batch_kernel(const CaseArgs* __restrict__ cases,
                                                                 int partial_stride) {
  __shared__ double2 wsum[4];
  const int j = blockIdx.x;
  const CaseArgs& c = cases[blockIdx.y];
  if ((int64_t)j + c.hist_cap < (int64_t)gridDim.x) return;  // uniform per block
  const double2* __restrict__ part = c.partial + (size_t)j * partial_stride;
  double sx = 0.0, sy = 0.0;
  for (int i = threadIdx.x; i < c.g.n_link_nodes; i += 256) {
    const double2 v = part[i];
    sx += v.x;
    sy += v.y;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sx += __shfl_xor(sx, off);
    sy += __shfl_xor(sy, off);
  }
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = make_double2(sx, sy);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double fx = (wsum[0].x + wsum[1].x) + (wsum[2].x + wsum[3].x);
    const double fy = (wsum[0].y + wsum[1].y) + (wsum[2].y + wsum[3].y);
    const int64_t s = (*c.dev_step + j) % c.hist_cap;
    c.hist[2 * s] = fx;
    c.hist[2 * s + 1] = fy;
  }
}

__global__ void advance_batch_kernel(const CaseArgs* __restrict__ cases, int ncases, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncases) return;
  const CaseArgs& c = cases[i];
  const int64_t base = *c.dev_step;
  const int b = *c.bad;
  if (b != INT_MAX) {
    if (*c.bad_step == 0) *c.bad_step = base + b + 1;
    *c.bad = INT_MAX;
  }
  *c.dev_step = base + count;
}

// Runs after force_reduce_kernel: advances the device step counter by
// `count` and turns the watchdog's ring slot into an absolute step.
__global__ void advance_kernel(int count, int64_t* dev_step, int* bad, int64_t* bad_step) {
  const int64_t base = *dev_step;
  const int b = *bad;
  if (b != INT_MAX) {
    if (*bad_step == 0) *bad_step = base + b + 1;
    *bad = INT_MAX;
  }
  *dev_step = base + count;
}

// Equilibrium of rho = 1 and the perturbed inlet velocity everywhere; with
// `rest_solid` (full-way bounce-back) solid nodes start at rest, f = w.
__global__ void init_eq_kernel(float* f, Geometry g, double u, double amp, int rest_solid) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx || y >= g.ny) return;
  const bool rest = rest_solid && (node_flags(g, x, y) & kSolid);
  const double v = amp * u * sin(2.0 * 3.14159265358979323846 * y / (double)(g.ny - 1));
  const double usq = 1.5 * (u * u + v * v);
  for (int k = 0; k < 9; ++k) {
    const double w = k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
    const double cu = CX[k] * u + CY[k] * v;
    f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x] = rest ? 0.0f : (float)(w * (cu * (3.0 + 4.5 * cu) - usq));
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
    r = 1.0f + (((h[0] + h[1]) + (h[2] + h[3])) + ((h[4] + h[5]) + (h[6] + h[7])) + h[8]);
    u = (((h[1] - h[3]) + (h[5] - h[7])) + (h[8] - h[6])) / r;
    v = (((h[2] - h[4]) + (h[5] - h[7])) + (h[6] - h[8])) / r;
  }
  if (rho) rho[i] = r;
  if (ux) ux[i] = u;
  if (uy) uy[i] = v;
}

__device__ __forceinline__ double weight(int k) {
  return k == 0 ? 4.0 / 9.0 : (k < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}

__global__ void pack_kernel(const float* __restrict__ f, Geometry g, void* dense, int dtype) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const double v = (double)f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x] + weight(k);
  const int64_t i = ((int64_t)k * g.ny + y) * g.nx + x;
  if (dtype == 0)
    ((float*)dense)[i] = (float)v;
  else
    ((double*)dense)[i] = v;
}

__global__ void unpack_kernel(const void* dense, int dtype, Geometry g, float* f) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y, k = blockIdx.z;
  if (x >= g.nx || y >= g.ny) return;
  const int64_t i = ((int64_t)k * g.ny + y) * g.nx + x;
  const double v = dtype == 0 ? (double)((const float*)dense)[i] : ((const double*)dense)[i];
  f[(int64_t)k * g.plane + (int64_t)y * g.pitch + x] = (float)(v - weight(k));
}

__global__ void fill_int_kernel(int* p, int value) { *p = value; }

typedef float float4v __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void copy_probe_kernel(const float4v* __restrict__ src,
                                                         float4v* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(src[i], dst + i);
}

constexpr Variant kVariants[] = {
    // name              tile_x tile_y vx remap nt steps sub
    {"v1_ty1_nt", 256, 1, 1, 0, 1, 1, 0},
    {"v1_ty1_xcd_nt", 256, 1, 1, 1, 1, 1, 0},
    {"v1_ty1", 256, 1, 1, 0, 0, 1, 0},
    {"v1_ty2_nt", 256, 2, 1, 0, 1, 1, 0},
    {"v2_ty1_nt", 512, 1, 2, 0, 1, 1, 0},
    {"v4_ty1_nt", 1024, 1, 4, 0, 1, 1, 0},
    {"v4_ty1_xcd_nt", 1024, 1, 4, 1, 1, 1, 0},
    {"v1_ty1_xrow_nt", 256, 1, 1, 2, 1, 1, 0},
    {"v2_ty1_xrow_nt", 512, 1, 2, 2, 1, 1, 0},
    {"v1_ty1_xcd", 256, 1, 1, 1, 0, 1, 0},
    {"t2_h4", kStrip2, 4, 1, 0, 0, 2, 2},
    {"t2_h6", kStrip2, 6, 1, 0, 0, 2, 2},
    {"t2_h8", kStrip2, 8, 1, 0, 0, 2, 2},
    {"t2_h8_nt", kStrip2, 8, 1, 0, 1, 2, 2},
    {"t2_h16", kStrip2, 16, 1, 0, 0, 2, 2},
    {"t2_h4_s4", kStrip2, 4, 1, 0, 0, 2, 4},
    {"t2_h6_s4", kStrip2, 6, 1, 0, 0, 2, 4},
    {"t3_h4_s4", kStrip3, 4, 1, 0, 0, 3, 4},
    {"t3_h6_s4", kStrip3, 6, 1, 0, 0, 3, 4},
    {"t3_h8_s4", kStrip3, 8, 1, 0, 0, 3, 4},
    {"t3_h12_s4", kStrip3, 12, 1, 0, 0, 3, 4},
    {"t3_h8_s8", kStrip3, 8, 1, 0, 0, 3, 8},
    {"t4_h8_s4", kStrip4, 8, 1, 0, 0, 4, 4},
    {"t4_h8_s8", kStrip4, 8, 1, 0, 0, 4, 8},
    {"t4_h12_s4", kStrip4, 12, 1, 0, 0, 4, 4},
    {"t4_h12_s12", kStrip4, 12, 1, 0, 0, 4, 12},
    {"t3_h8_s2", kStrip3, 8, 1, 0, 0, 3, 2},
    {"t4_h8_s2", kStrip4, 8, 1, 0, 0, 4, 2},
    {"t2_h4_u1", kStrip2, 4, 1, 0, 0, 2, 1, 1},
    {"t4_h16u_s8", kStrip4, 16, 1, 0, 0, 4, 8, 0, 2},
    {"t4_h8u_s8", kStrip4, 8, 1, 0, 0, 4, 8, 0, 2},
    {"t4_h12u_s12", kStrip4, 12, 1, 0, 0, 4, 12, 0, 2},
    {"t4_h24u_s8", kStrip4, 24, 1, 0, 0, 4, 8, 0, 2},
    {"t3_h16u_s2", kStrip3, 16, 1, 0, 0, 3, 2, 0, 2},
    {"t4_h16u_s2", kStrip4, 16, 1, 0, 0, 4, 2, 0, 2},
    {"t4_h12u_s6", kStrip4, 12, 1, 0, 0, 4, 6, 0, 2},
    {"t4_h10u_s10", kStrip4, 10, 1, 0, 0, 4, 10, 0, 2},
    {"t4_h14u_s14", kStrip4, 14, 1, 0, 0, 4, 14, 0, 2},
    {"t3_h10u_s2", kStrip3, 10, 1, 0, 0, 3, 2, 0, 2},
    {"t3_h12u_s2", kStrip3, 12, 1, 0, 0, 3, 2, 0, 2},
    {"t2_h6_u1", kStrip2, 6, 1, 0, 0, 2, 1, 1},
    {"t2_h8_u1", kStrip2, 8, 1, 0, 0, 2, 1, 1},
};

}  // namespace

int num_variants() { return (int)(sizeof(kVariants) / sizeof(kVariants[0])); }
const Variant& variant(int v) { return kVariants[v - 1]; }

// Measured on the MI355X (BGK, D2Q9 cylinder channels and one x-periodic
// slab; MRT on the paper's lattice and the closure window): below 2^18 nodes
// one launch per step, with cached stores and each XCD on its own band of
// rows, is fastest (4.2 us per step at 86 k nodes against 4.7 us for two
// steps); from 2^18 two steps with one-row boundary pieces that load all
// their rows first (6.1 against 6.3 us per step at 320 k nodes, 6.3 against
// 7.1 us at 458 k), where the deeper kernels' boundary chains still set the
// launch time.  From 2^20 nodes more fused steps win: at 1.4 M nodes three steps with 2-row boundary
// pieces and 16-row interior segments storing rows as they are made (154 k
// MLUPS against 144 k with 8-row segments holding them, 132 k for four and
// 108 k for two steps), from
// 2.8 M four steps with 8-row pieces and 16-row interior segments that store
// each row as it is made (178 k on the 2.8 M slab, 193 k at 5.5 M, 220 k at
// 22 M, against 165 k, 191 k and 209 k with 8-row segments holding their
// outputs; one step per launch gives 82 k at 22 M).  Longer
// boundary pieces recompute fewer rows but lengthen the serial chain of each
// boundary wave, which only long launches hide.  On the row-interleaved
// state 10-row segments with 10-row pieces win from 2^21 nodes (233 k MLUPS
// at 22 M, tied with 12-row ones, against 223 k for 16-row segments with
// 8-row pieces; 199 k against 194 k and 191 k at 5.5 M; 188 k against 183 k
// on the 2.8 M slab).  For two steps the row-interleaved state favours 8-row
// interior segments with the same one-row boundary pieces (6.0 against 6.3 us
// per step on the 458 k-node closure window, 5.5 against 5.9 at 320 k; 12 and
// 16 rows lose).
int default_variant(int64_t nodes) {
  const char* want = nodes >= ((int64_t)1 << 21)   ? "t4_h10u_s10"
                     : nodes >= ((int64_t)1 << 20) ? "t3_h16u_s2"
                     : nodes >= ((int64_t)1 << 18) ? "t2_h8_u1"
                                                   : "v1_ty1_xcd";
  for (int v = 1; v <= num_variants(); ++v)
    if (std::strcmp(kVariants[v - 1].name, want) == 0) return v;
  return 1;
}

hipError_t launch_step_batch(const CaseArgs* cases, const int2* tiles, int ntiles, int cur, int slot,
                             int partial_stride, int v, hipStream_t s) {
  const Variant& var = variant(v);
  const dim3 grid((unsigned)ntiles), block(256);
#define LBM_CASE(TY, VX, NT)                                                                   \
  if (var.tile_y == TY && var.vx == VX && var.nontemporal == NT) {                              \
    hipLaunchKernelGGL((step_batch_kernel<TY, VX, NT>), grid, block, 0, s, cases, tiles, cur,   \
                       slot, partial_stride);                                                   \
    return hipGetLastError();                                                                   \
  }
  LBM_CASE(1, 1, 1)
  LBM_CASE(1, 1, 0)
  LBM_CASE(2, 1, 1)
  LBM_CASE(1, 2, 1)
  LBM_CASE(1, 4, 1)
#undef LBM_CASE
  return hipErrorInvalidValue;
}

// Multi-step variants the ensemble runs (instantiated below).
#define LBM_TB_LIST(X) X(8, 2, 3, 0) X(8, 4, 3, 0) X(8, 2, 4, 0) X(8, 4, 4, 0) X(8, 8, 4, 0) X(16, 8, 4, 2) \
  X(16, 2, 3, 2) X(10, 10, 4, 2)

bool multistep_batch_supported(int v) {
  if (v < 1 || v > num_variants()) return false;
  const Variant& var = variant(v);
  if (var.nontemporal || var.steps < 3) return false;
#define LBM_TB_HAS(H, SUB, S, STREAM) \
  if (var.tile_y == H && var.sub == SUB && var.steps == S && var.stream == STREAM) return true;
  LBM_TB_LIST(LBM_TB_HAS)
#undef LBM_TB_HAS
  return false;
}

hipError_t launch_multistep_batch(const CaseArgs* cases, const int2* gen_tasks, int n_gen, const int2* bulk_tasks,
                                  int n_bulk, int cur, int slot, int partial_stride, int v, hipStream_t s) {
  if (!multistep_batch_supported(v)) return hipErrorInvalidValue;
  const Variant& var = variant(v);
  const dim3 grid((unsigned)((n_gen + n_bulk + 3) / 4)), block(256);
#define LBM_TB_LAUNCH(H, SUB, S, STREAM)                                                           \
  if (var.tile_y == H && var.sub == SUB && var.steps == S && var.stream == STREAM) {                 \
    hipLaunchKernelGGL((multistep_batch_kernel<false, H, SUB, S, STREAM>), grid, block, 0, s, cases,  \
                       gen_tasks, n_gen, bulk_tasks, n_bulk, cur, slot, partial_stride);             \
    return hipGetLastError();                                                                        \
  }
  LBM_TB_LIST(LBM_TB_LAUNCH)
#undef LBM_TB_LAUNCH
  return hipErrorInvalidValue;
}
#undef LBM_TB_LIST

hipError_t launch_force_reduce_batch(const CaseArgs* cases, int ncases, int count, int partial_stride,
                                     hipStream_t s) {
  hipLaunchKernelGGL(force_reduce_batch_kernel, dim3(count, ncases), dim3(256), 0, s, cases,
                     partial_stride);
  hipLaunchKernelGGL(advance_batch_kernel, dim3((ncases + 63) / 64), dim3(64), 0, s, cases, ncases,
                     count);
  return hipGetLastError();
}

bool step_fuses_closure(int v, int k) { return k == 2 && variant(v).steps == 2; }

hipError_t launch_step(const StepArgs& a, int v, hipStream_t s) {
  const Variant& var = variant(v);
  if (a.ev.blocks > 0 && !step_fuses_closure(v, var.steps)) return hipErrorInvalidValue;
  if (var.steps == 2) {
    const int per = (var.tile_y + var.sub - 1) / var.sub;
    const int blocks = a.ev.blocks + (a.n_gen * per + 3) / 4 + (a.t.ntx * a.t.nty + 3) / 4;
    const dim3 grid((unsigned)blocks), block(256);
    const size_t lds = a.ev.blocks > 0 ? closure_lds_bytes() : 0;
#define LBM_T2(NT, H, SUB, UNR)                                                              \
  if (var.nontemporal == NT && var.tile_y == H && var.sub == SUB && var.unrolled == UNR) {   \
    if (a.ev.blocks > 0)                                                                     \
      hipLaunchKernelGGL((step2_kernel<NT, H, SUB, UNR, true>), grid, block, lds, s, a);     \
    else                                                                                     \
      hipLaunchKernelGGL((step2_kernel<NT, H, SUB, UNR, false>), grid, block, 0, s, a);      \
    return hipGetLastError();                                                                \
  }
    LBM_T2(false, 4, 2, 0)
    LBM_T2(false, 6, 2, 0)
    LBM_T2(false, 8, 2, 0)
    LBM_T2(true, 8, 2, 0)
    LBM_T2(false, 16, 2, 0)
    LBM_T2(false, 4, 4, 0)
    LBM_T2(false, 6, 4, 0)
    LBM_T2(false, 4, 1, 1)
    LBM_T2(false, 6, 1, 1)
    LBM_T2(false, 8, 1, 1)
#undef LBM_T2
    return hipErrorInvalidValue;
  }
  if (var.steps >= 3) {
    const int per = (var.tile_y + var.sub - 1) / var.sub;
    const int blocks = (a.n_gen * per + 3) / 4 + (a.t.ntx * a.t.nty + 3) / 4;
    const dim3 grid((unsigned)blocks), block(256);
#define LBM_TN(NT, H, SUB, S, STREAM)                                                         \
  if (var.nontemporal == NT && var.tile_y == H && var.sub == SUB && var.steps == S &&           \
      var.stream == STREAM) {                                                                    \
    if (a.p.mrt)                                                                                 \
      hipLaunchKernelGGL((multistep_kernel<NT, H, SUB, S, kMrt, STREAM>), grid, block, 0, s, a); \
    else                                                                                         \
      hipLaunchKernelGGL((multistep_kernel<NT, H, SUB, S, kBgk, STREAM>), grid, block, 0, s, a); \
    return hipGetLastError();                                                                    \
  }
    LBM_TN(false, 4, 4, 3, 0)
    LBM_TN(false, 6, 4, 3, 0)
    LBM_TN(false, 8, 4, 3, 0)
    LBM_TN(false, 12, 4, 3, 0)
    LBM_TN(false, 8, 8, 3, 0)
    LBM_TN(false, 8, 4, 4, 0)
    LBM_TN(false, 8, 8, 4, 0)
    LBM_TN(false, 12, 4, 4, 0)
    LBM_TN(false, 12, 12, 4, 0)
    LBM_TN(false, 8, 2, 3, 0)
    LBM_TN(false, 8, 2, 4, 0)
    LBM_TN(false, 16, 8, 4, 2)
    LBM_TN(false, 8, 8, 4, 2)
    LBM_TN(false, 12, 12, 4, 2)
    LBM_TN(false, 24, 8, 4, 2)
    LBM_TN(false, 16, 2, 3, 2)
    LBM_TN(false, 16, 2, 4, 2)
    LBM_TN(false, 12, 6, 4, 2)
    LBM_TN(false, 10, 10, 4, 2)
    LBM_TN(false, 14, 14, 4, 2)
    LBM_TN(false, 10, 2, 3, 2)
    LBM_TN(false, 12, 2, 3, 2)
#undef LBM_TN
    return hipErrorInvalidValue;
  }
  const dim3 grid((unsigned)(a.t.ntx * a.t.nty)), block(256);
#define LBM_CASE(TY, VX, NT)                                                       \
  if (var.tile_y == TY && var.vx == VX && var.nontemporal == NT) {                  \
    hipLaunchKernelGGL((step_kernel<TY, VX, NT>), grid, block, 0, s, a);            \
    return hipGetLastError();                                                       \
  }
  LBM_CASE(1, 1, 1)
  LBM_CASE(1, 1, 0)
  LBM_CASE(2, 1, 1)
  LBM_CASE(1, 2, 1)
  LBM_CASE(1, 4, 1)
#undef LBM_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_force_reduce(const double2* partials, int nnodes, int count, double* hist,
                               int64_t cap, int64_t* dev_step, int* bad, int64_t* bad_step,
                               hipStream_t s) {
  hipLaunchKernelGGL(force_reduce_kernel, dim3(count), dim3(256), 0, s, partials, nnodes, hist, cap,
                     (const int64_t*)dev_step);
  hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(1), 0, s, count, dev_step, bad, bad_step);
  return hipGetLastError();
}

hipError_t launch_init_equilibrium(float* f, const Geometry& g, double u, double amp, bool rest_solid,
                                   hipStream_t s) {
  hipLaunchKernelGGL(init_eq_kernel, dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s, f, g, u, amp,
                     (int)rest_solid);
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

hipError_t launch_copy_probe(void* dst, const void* src, int64_t nbytes, hipStream_t s) {
  const int64_t n = nbytes / 16;
  hipLaunchKernelGGL(copy_probe_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     (const float4v*)src, (float4v*)dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int value, hipStream_t s) {
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, s, p, value);
  return hipGetLastError();
}

}  // namespace lbm
