// Host runtime of liblbm.so: parameter validation, geometry, device state,
// step scheduling and the C ABI of include/lbm.h.
#include "../../include/lbm.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_internal.h"

namespace {

thread_local std::string g_err;

lbm_status fail(lbm_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
lbm_status fail(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? LBM_ERR_OOM : LBM_ERR_HIP, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

// Table 1 with k = i - 1 (host copy for geometry and link flags).
const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

bool solid_at(const lbm_params& p, int x, int y) {
  if (p.diameter <= 0) return false;
  const int64_t dx = 2LL * x - p.cx2, dy = 2LL * y - p.cy2;
  return dx * dx + dy * dy <= (int64_t)p.diameter * p.diameter;
}

double wall_u(double v, double u_in) { return std::isnan(v) ? u_in : v; }

}  // namespace

namespace lbm {

lbm_status set_error(lbm_status s, const char* msg) { return fail(s, "%s", msg); }

// Sec. 2.4, link-wise approach: the wall cuts the link from fluid node
// (x, y) into the solid (along -c_k for pull direction k) at a fraction q of
// its length.  With the disk's circle in doubled coordinates, X = 2x - cx2,
// Y = 2y - cy2, the cut solves (X - 2q c_kx)^2 + (Y - 2q c_ky)^2 = D^2; its
// smaller root lies in (0, 1].  Where q < 1/2 needs the fluid node on the
// far side (x + c_k) and that node is not fluid, the link falls back to
// q = 1/2 (half-way bounce-back).
double link_fraction(const lbm_params& p, int x, int y, int k) {
  const double X = 2.0 * x - p.cx2, Y = 2.0 * y - p.cy2, D = p.diameter;
  const double dx = -CX[k], dy = -CY[k];
  const double a = 4.0 * (dx * dx + dy * dy), b = 4.0 * (X * dx + Y * dy), c = X * X + Y * Y - D * D;
  const double disc = std::max(0.0, b * b - 4.0 * a * c);
  double q = (-b - std::sqrt(disc)) / (2.0 * a);
  q = std::min(1.0, std::max(1e-12, q));
  const int xb = x + CX[k], yb = y + CY[k];
  const bool behind_fluid = xb >= 0 && xb < p.nx && yb >= 0 && yb < p.ny && !solid_at(p, xb, yb);
  if (q < 0.5 && !behind_fluid) q = 0.5;
  return q;
}

lbm_status build_geometry(const lbm_params* p, HostGeometry* out) {
  Geometry& g = out->g;
  g = Geometry{};
  g.nx = p->nx;
  g.ny = p->ny;
  // Row-interleaved storage: row y holds the nine populations' rows one
  // after another (population k of node (x, y) at k * plane + y * pitch + x,
  // plane = one row padded to 64 floats, pitch = nine of them), so the rows a
  // wave reads and writes lie together instead of in nine planes a lattice
  // apart: 4.5 % faster at D = 160 and 5 % on the paper's E1 lattice than
  // nine separate planes (bit-identical results; the kernels only see the
  // two strides).
  g.plane = (int64_t)(p->nx + 63) / 64 * 64;
  g.pitch = (int)(9 * g.plane);
  if ((int64_t)p->ny * g.pitch + 9 * g.plane >= (int64_t)INT_MAX)
    return fail(LBM_ERR_INVALID_ARG, "lattice of %d x %d exceeds the 32-bit offsets of the kernels", p->nx, p->ny);
  out->flags.clear();
  out->link_index.clear();
  // cylinder rectangle: solid nodes plus one ring of fluid neighbours
  if (p->diameter > 0) {
    int x0 = INT_MAX, x1 = -1, y0 = INT_MAX, y1 = -1;
    for (int y = 0; y < p->ny; ++y)
      for (int x = 0; x < p->nx; ++x)
        if (solid_at(*p, x, y)) {
          x0 = std::min(x0, x);
          x1 = std::max(x1, x);
          y0 = std::min(y0, y);
          y1 = std::max(y1, y);
        }
    if (x1 >= 0) {
      g.rx0 = x0 - 1;
      g.ry0 = y0 - 1;
      g.rw = x1 - x0 + 3;
      g.rh = y1 - y0 + 3;
      out->flags.resize((size_t)g.rw * g.rh);
      out->link_index.assign((size_t)g.rw * g.rh, -1);
      for (int j = 0; j < g.rh; ++j)
        for (int i = 0; i < g.rw; ++i) {
          const int x = g.rx0 + i, y = g.ry0 + j;
          uint16_t f = 0;
          if (solid_at(*p, x, y)) {
            f = kSolid;
          } else {
            for (int k = 1; k < 9; ++k)
              if (solid_at(*p, x - CX[k], y - CY[k])) f |= (uint16_t)(1u << k);
          }
          out->flags[(size_t)j * g.rw + i] = f;
          if (f >> 1) out->link_index[(size_t)j * g.rw + i] = g.n_link_nodes++;
        }
      if (p->bounce == LBM_BOUNCE_INTERP) {
        out->q.assign((size_t)g.n_link_nodes * 8, 0.5f);
        for (int j = 0; j < g.rh; ++j)
          for (int i = 0; i < g.rw; ++i) {
            const int32_t idx = out->link_index[(size_t)j * g.rw + i];
            if (idx < 0) continue;
            const int x = g.rx0 + i, y = g.ry0 + j;
            for (int k = 1; k < 9; ++k)
              if ((out->flags[(size_t)j * g.rw + i] >> k) & 1)
                out->q[(size_t)idx * 8 + k - 1] = (float)link_fraction(*p, x, y, k);
          }
      }
    }
  }
  return LBM_OK;
}

Physics make_physics(const lbm_params* p) {
  Physics ph{};
  ph.omega = (float)(1.0 / lbm_params_tau(p));
  ph.u_in = (float)p->u_in;
  ph.u_top = (float)wall_u(p->u_wall_top, p->u_in);
  ph.u_bot = (float)wall_u(p->u_wall_bottom, p->u_in);
  ph.wall = p->wall;
  ph.outlet_mode = p->outlet_mode;
  ph.x_periodic = p->x_periodic;
  ph.mrt = p->collision == LBM_COLLISION_MRT;
  ph.interp_bb = p->bounce == LBM_BOUNCE_INTERP && p->diameter > 0;
  ph.full_bb = p->bounce == LBM_BOUNCE_FULLWAY && p->diameter > 0;
  auto rate = [&](int i) { return (float)(p->s_rates[i] > 0 ? p->s_rates[i] : 1.0 / lbm_params_tau(p)); };
  ph.s_e = rate(1);
  ph.s_eps = rate(2);
  ph.s_qx = rate(4);
  ph.s_qy = rate(6);
  ph.s_pxx = rate(7);
  ph.s_pxy = rate(8);
  return ph;
}

void tiling_for_variant(const Geometry& g, int v, Tiling* t) {
  const Variant& var = variant(v);
  t->tile_x = var.tile_x;
  t->tile_y = var.tile_y;
  t->ntx = (g.nx + t->tile_x - 1) / t->tile_x;
  t->nty = (g.ny + t->tile_y - 1) / t->tile_y;
  t->remap_xcd = var.remap_xcd;
}

}  // namespace lbm

struct lbm_ctx {
  lbm_params p{};
  double tau = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  lbm::Geometry geo{};
  lbm::Physics phys{};
  lbm::Tiling tiling{};
  int variant = 1;
  float* buf[2] = {nullptr, nullptr};
  int cur = 0;
  uint16_t* d_flags = nullptr;
  int32_t* d_link_index = nullptr;
  float* d_q = nullptr;
  double2* d_partials = nullptr;
  // two-step variants: segments that need the boundary code (seg * ntx + strip)
  int* d_gen = nullptr;
  int n_gen = 0;
  double* d_hist = nullptr;
  int64_t* d_step = nullptr;
  int* d_bad = nullptr;
  int64_t* d_bad_step = nullptr;
  int64_t step = 0;
  int pending = 0;
  // graph replay of kRing steps; graph[c | r << 1] starts from buf[c] with
  // d_resid[r] the learned-closure residuals in use
  int use_graphs = 1;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  int graph_flip[4] = {0, 0, 0, 0};  // 1: the graph leaves the state in the other buffer (odd launches)
  int resid_flip[4] = {0, 0, 0, 0};  // 1: it leaves the other residual buffer in use (odd evaluations)
  // learned closure
  const lbm_mlp* mlp = nullptr;
  int closure_mask = 7;
  float closure_beta = 1.0f;
  int closure_taper = 0;
  float closure_limit = 0.0f;
  int closure_outlet_taper = 0;
  int closure_outlet_neutral = 0;
  float* d_bias = nullptr;  // per-node fixed part of the residual [nb][3], or null
  int closure_interval = 1;
  float* d_norm = nullptr;
  // d_resid[rc] are the residuals the steps apply; an evaluation writes the
  // next ones into d_resid[rc ^ 1], in the launch that starts at its step
  // (two-step kernels) or in a closure launch just before it.
  float* d_resid[2] = {nullptr, nullptr};
  int rc = 1;
  float* d_resid_q = nullptr;  // lbm_closure_residuals
};

extern "C" {

void lbm_params_init(lbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->struct_size = (int32_t)sizeof(lbm_params);
  p->u_in = 0.1;
  p->re = 100.0;
  p->tau = 0.0;
  p->wall = LBM_WALL_FREE_SLIP;
  p->outlet_mode = LBM_OUTLET_COPY_ALL;
  p->u_wall_top = NAN;
  p->u_wall_bottom = NAN;
  p->perturb_amp = 1e-3;
  p->hist_capacity = 1 << 20;
  p->collision = LBM_COLLISION_BGK;
  const double paper_rates[9] = {1.0, 1.1, 1.1, 1.0, 1.1, 1.0, 1.1, 0.0, 0.0};  // Sec. 2.1
  for (int i = 0; i < 9; ++i) p->s_rates[i] = paper_rates[i];
}

double lbm_params_tau(const lbm_params* p) {
  if (!p) return NAN;
  if (p->tau > 0) return p->tau;
  const double nu = p->u_in * p->diameter / p->re;  // Eq. 16
  return 3.0 * nu + 0.5;                            // Eq. 17
}

lbm_status lbm_validate_params(const lbm_params* p) {
  if (!p) return fail(LBM_ERR_INVALID_ARG, "params is NULL");
  if (p->struct_size != (int32_t)sizeof(lbm_params))
    return fail(LBM_ERR_INVALID_ARG, "struct_size %d != %d (call lbm_params_init)", p->struct_size,
                (int)sizeof(lbm_params));
  if (p->nx < 3 || p->ny < 3) return fail(LBM_ERR_INVALID_ARG, "nx, ny must be >= 3 (got %d, %d)", p->nx, p->ny);
  if (p->wall < LBM_WALL_FREE_SLIP || p->wall > LBM_WALL_MOVING_BB)
    return fail(LBM_ERR_INVALID_ARG, "unknown wall mode %d", p->wall);
  if (p->outlet_mode != LBM_OUTLET_COPY_ALL && p->outlet_mode != LBM_OUTLET_COPY_UNKNOWN)
    return fail(LBM_ERR_INVALID_ARG, "unknown outlet mode %d", p->outlet_mode);
  if (p->x_periodic != 0 && p->x_periodic != 1) return fail(LBM_ERR_INVALID_ARG, "x_periodic must be 0 or 1");
  if (p->collision != LBM_COLLISION_BGK && p->collision != LBM_COLLISION_MRT)
    return fail(LBM_ERR_INVALID_ARG, "unknown collision %d", p->collision);
  if (p->bounce != LBM_BOUNCE_HALFWAY && p->bounce != LBM_BOUNCE_INTERP && p->bounce != LBM_BOUNCE_FULLWAY)
    return fail(LBM_ERR_INVALID_ARG, "unknown bounce-back mode %d", p->bounce);
  if (p->collision == LBM_COLLISION_MRT)
    for (int i : {1, 2, 4, 6, 7, 8}) {
      const double s = p->s_rates[i];
      if ((i == 7 || i == 8) && s <= 0) continue;  // 1/tau
      if (!(s > 0.0 && s < 2.0)) return fail(LBM_ERR_INVALID_ARG, "MRT rate s_rates[%d] = %g outside (0, 2)", i, s);
    }
  if (!(p->u_in >= 0.0 && p->u_in < 1.0 / std::sqrt(3.0)))
    return fail(LBM_ERR_INVALID_ARG, "u_in = %g outside [0, 1/sqrt(3))", p->u_in);
  if (p->tau <= 0 && !(p->re > 0)) return fail(LBM_ERR_INVALID_ARG, "re must be > 0 when tau is derived");
  const double tau = lbm_params_tau(p);
  if (!(tau > 0.5) || !std::isfinite(tau)) return fail(LBM_ERR_INVALID_ARG, "tau = %g must be > 1/2", tau);
  for (double uw : {p->u_wall_top, p->u_wall_bottom})
    if (!std::isnan(uw) && !(std::fabs(uw) < 1.0 / std::sqrt(3.0)))
      return fail(LBM_ERR_INVALID_ARG, "wall velocity %g out of range", uw);
  if (p->diameter < 0) return fail(LBM_ERR_INVALID_ARG, "diameter must be >= 0");
  if (p->diameter > 0) {
    // bounding box of the disk in doubled coordinates: [c - D, c + D]
    const int64_t xlo = p->cx2 - p->diameter, xhi = p->cx2 + p->diameter;
    const int64_t ylo = p->cy2 - p->diameter, yhi = p->cy2 + p->diameter;
    // 2-node margin: every node within 2 of a solid node lies inside [1, n-2]
    if (xlo < 2 * 3 || xhi > 2 * ((int64_t)p->nx - 4) || ylo < 2 * 3 || yhi > 2 * ((int64_t)p->ny - 4))
      return fail(LBM_ERR_INVALID_ARG, "cylinder must stay at least 2 nodes away from every edge");
  }
  if (p->hist_capacity < 1) return fail(LBM_ERR_INVALID_ARG, "hist_capacity must be >= 1");
  if (!std::isfinite(p->perturb_amp)) return fail(LBM_ERR_INVALID_ARG, "perturb_amp must be finite");
  return LBM_OK;
}

lbm_status lbm_geometry(const lbm_params* p, uint8_t* solid_mask, int64_t* n_solid,
                        int64_t* n_boundary_nodes, int64_t* n_links) {
  if (!p || p->nx < 1 || p->ny < 1) return fail(LBM_ERR_INVALID_ARG, "bad params");
  int64_t ns = 0, nb = 0, nl = 0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      const bool s = solid_at(*p, x, y);
      if (solid_mask) solid_mask[(int64_t)y * p->nx + x] = s ? 1 : 0;
      if (s) {
        ++ns;
        continue;
      }
      int links = 0;
      for (int k = 1; k < 9; ++k) links += solid_at(*p, x + CX[k], y + CY[k]);
      nl += links;
      nb += links > 0;
    }
  if (n_solid) *n_solid = ns;
  if (n_boundary_nodes) *n_boundary_nodes = nb;
  if (n_links) *n_links = nl;
  return LBM_OK;
}

int32_t lbm_num_variants(void) { return lbm::num_variants(); }

int32_t lbm_get_variant(const lbm_ctx* c) { return c ? c->variant : 0; }

const char* lbm_variant_name(int32_t v) {
  if (v < 1 || v > lbm::num_variants()) return "";
  return lbm::variant(v).name;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

lbm_status set_tiling(lbm_ctx* c, int v) {
  lbm::Tiling t;
  lbm::tiling_for_variant(c->geo, v, &t);
  if (lbm::variant(v).steps >= 2) {
    std::vector<int> gen;
    for (int seg = 0; seg < t.nty; ++seg)
      for (int strip = 0; strip < t.ntx; ++strip)
        if (!lbm::interior_segment(c->geo, t, c->p.x_periodic != 0, strip, seg)) gen.push_back(seg * t.ntx + strip);
    int* d = nullptr;
    HIP_TRY(hipMalloc(&d, sizeof(int) * gen.size()));
    const hipError_t e = hipMemcpy(d, gen.data(), sizeof(int) * gen.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(d);
      return fail(LBM_ERR_HIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    (void)hipFree(c->d_gen);
    c->d_gen = d;
    c->n_gen = (int)gen.size();
  }
  c->tiling = t;
  c->variant = v;
  return LBM_OK;
}

// force contributions per step: one per link node, at least one row entry
int slots_of(const lbm_ctx* c) { return std::max(1, c->geo.n_link_nodes); }

lbm_status flush(lbm_ctx* c) {
  if (c->pending == 0) return LBM_OK;
  HIP_TRY(lbm::launch_force_reduce(c->d_partials, slots_of(c), c->pending, c->d_hist,
                                   c->p.hist_capacity, c->d_step, c->d_bad, c->d_bad_step, c->stream));
  c->pending = 0;
  return LBM_OK;
}

void drop_graphs(lbm_ctx* c) {
  for (int i = 0; i < 4; ++i)
    if (c->graph[i]) {
      (void)hipGraphExecDestroy(c->graph[i]);
      c->graph[i] = nullptr;
    }
}

void free_ctx(lbm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  drop_graphs(c);
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  (void)hipFree(c->buf[0]);
  (void)hipFree(c->buf[1]);
  (void)hipFree(c->d_flags);
  (void)hipFree(c->d_link_index);
  (void)hipFree(c->d_q);
  (void)hipFree(c->d_partials);
  (void)hipFree(c->d_gen);
  (void)hipFree(c->d_hist);
  (void)hipFree(c->d_step);
  (void)hipFree(c->d_bad);
  (void)hipFree(c->d_bad_step);
  (void)hipFree(c->d_norm);
  (void)hipFree(c->d_resid[0]);
  (void)hipFree(c->d_resid[1]);
  (void)hipFree(c->d_resid_q);
  (void)hipFree(c->d_bias);
  delete c;
}

lbm_status check_ctx(lbm_ctx* c) {
  if (!c) return fail(LBM_ERR_INVALID_ARG, "context is NULL");
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_create(const lbm_params* p, void* stream, lbm_ctx** out) {
  if (!out) return fail(LBM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  lbm_status st = lbm_validate_params(p);
  if (st != LBM_OK) return st;
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->tau = lbm_params_tau(p);
  c->stream = (hipStream_t)stream;
  {
    const hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) {
      delete c;
      return fail(LBM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    }
  }
  lbm::HostGeometry hg;
  st = lbm::build_geometry(p, &hg);
  if (st != LBM_OK) {
    delete c;
    return st;
  }
  c->geo = hg.g;
  lbm::Geometry& g = c->geo;
  const std::vector<uint16_t>& flags = hg.flags;
  const std::vector<int32_t>& link_index = hg.link_index;
  c->phys = lbm::make_physics(p);

  if ((st = set_tiling(c, lbm::default_variant((int64_t)p->nx * p->ny))) != LBM_OK) {
    free_ctx(c);
    return st;
  }

#define CREATE_TRY(call)            \
  do {                              \
    lbm_status s_ = [&]() -> lbm_status { HIP_TRY(call); return LBM_OK; }(); \
    if (s_ != LBM_OK) {             \
      free_ctx(c);                  \
      return s_;                    \
    }                               \
  } while (0)

  const size_t fbytes = (size_t)lbm::state_floats(g) * sizeof(float);
  CREATE_TRY(hipMalloc(&c->buf[0], fbytes));
  CREATE_TRY(hipMalloc(&c->buf[1], fbytes));
  CREATE_TRY(hipMemsetAsync(c->buf[0], 0, fbytes, c->stream));
  CREATE_TRY(hipMemsetAsync(c->buf[1], 0, fbytes, c->stream));
  if (!flags.empty()) {
    CREATE_TRY(hipMalloc(&c->d_flags, flags.size() * sizeof(uint16_t)));
    CREATE_TRY(hipMemcpyAsync(c->d_flags, flags.data(), flags.size() * sizeof(uint16_t),
                              hipMemcpyHostToDevice, c->stream));
  }
  if (!link_index.empty()) {
    CREATE_TRY(hipMalloc(&c->d_link_index, link_index.size() * sizeof(int32_t)));
    CREATE_TRY(hipMemcpyAsync(c->d_link_index, link_index.data(), link_index.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, c->stream));
  }
  if (!hg.q.empty()) {
    CREATE_TRY(hipMalloc(&c->d_q, hg.q.size() * sizeof(float)));
    CREATE_TRY(hipMemcpyAsync(c->d_q, hg.q.data(), hg.q.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
  }
  g.flags = c->d_flags;
  g.link_index = c->d_link_index;
  g.q = c->d_q;
  {
    const size_t bytes = sizeof(double2) * (size_t)slots_of(c) * lbm::kRing;
    CREATE_TRY(hipMalloc(&c->d_partials, bytes));
    // without any link node the single entry per step stays zero
    CREATE_TRY(hipMemsetAsync(c->d_partials, 0, bytes, c->stream));
  }
  CREATE_TRY(hipMalloc(&c->d_hist, sizeof(double) * 2 * (size_t)p->hist_capacity));
  CREATE_TRY(hipMemsetAsync(c->d_hist, 0, sizeof(double) * 2 * (size_t)p->hist_capacity, c->stream));
  CREATE_TRY(hipMalloc(&c->d_step, sizeof(int64_t)));
  CREATE_TRY(hipMalloc(&c->d_bad_step, sizeof(int64_t)));
  CREATE_TRY(hipMalloc(&c->d_bad, sizeof(int)));
  CREATE_TRY(hipMemsetAsync(c->d_step, 0, sizeof(int64_t), c->stream));
  CREATE_TRY(hipMemsetAsync(c->d_bad_step, 0, sizeof(int64_t), c->stream));
  CREATE_TRY(lbm::launch_fill_int(c->d_bad, INT_MAX, c->stream));
  CREATE_TRY(lbm::launch_init_equilibrium(c->buf[0], g, p->u_in, p->perturb_amp, c->phys.full_bb != 0,
                                          c->stream));
  CREATE_TRY(hipStreamSynchronize(c->stream));
#undef CREATE_TRY
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) { free_ctx(ctx); }

lbm_status lbm_set_variant(lbm_ctx* c, int32_t v) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (v == 0) v = lbm::default_variant((int64_t)c->p.nx * c->p.ny);
  if (v < 1 || v > lbm::num_variants()) return fail(LBM_ERR_INVALID_ARG, "variant %d out of range", v);
  lbm_status st = flush(c);
  if (st != LBM_OK) return st;
  drop_graphs(c);
  return set_tiling(c, v);
}

}  // extern "C"

namespace {

// The learned closure is evaluated on the state before each step whose index
// t is a multiple of its interval; its residuals take effect at step
// t + interval (until then the previous evaluation's apply).  The
// one-interval lag lets the network run in the same launch as the steps it
// does not feed.
bool closure_due(const lbm_ctx* c) { return c->mlp && c->step % c->closure_interval == 0; }

// Steps t .. t+k-1 share one launch only if no closure evaluation falls
// strictly inside them (an evaluation precedes each step whose index is a
// multiple of the interval and reads the state before it); every level of a
// multi-step launch applies the residuals held since the last evaluation, as
// k one-step launches would.
bool closure_allows(const lbm_ctx* c, int k) {
  if (!c->mlp) return true;
  return c->closure_interval - c->step % c->closure_interval >= k;
}

// Steps of the next launch, with `left` steps still to go: the variant's two,
// three or four when they fit in the force ring and between closure
// evaluations, else one.
int group(const lbm_ctx* c, int64_t left) {
  const int s = lbm::variant(c->variant).steps;
  if (s >= 2 && left >= s && c->pending + s <= lbm::kRing && closure_allows(c, s)) return s;
  return 1;
}

// Enqueues k = 1 to 4 steps (k > 1 only as group() allows) on stream s,
// buffers by c->cur and ring slots from c->pending, and advances the
// host-side bookkeeping; folds the ring when it is full.  One launch always
// moves the state from buf[cur] to buf[cur ^ 1].
lbm_status enqueue_step(lbm_ctx* c, hipStream_t s, int k = 1) {
  lbm::StepArgs a{};
  a.g = c->geo;
  a.p = c->phys;
  a.t = c->tiling;
  a.bad = c->d_bad;
  a.A = c->buf[c->cur];
  a.B = c->buf[c->cur ^ 1];
  a.slot = c->pending;
  a.partial = c->d_partials + (size_t)c->pending * slots_of(c);
  int v = c->variant;
  if (k >= 2) {
    a.partial2 = a.partial + slots_of(c);
    a.partial3 = k >= 3 ? a.partial2 + slots_of(c) : nullptr;
    a.partial4 = k >= 4 ? a.partial3 + slots_of(c) : nullptr;
    a.gen = c->d_gen;
    a.n_gen = c->n_gen;
  } else if (lbm::variant(v).steps != 1) {
    v = 1;  // a single step of a multi-step variant: the plain one-step kernel
    lbm::tiling_for_variant(c->geo, v, &a.t);
  }
  if (c->mlp) {
    if (closure_due(c)) {
      // the previous evaluation's residuals now apply; the network reads the
      // state before this launch and writes the next ones
      c->rc ^= 1;
      const lbm::MlpDevice md = lbm::mlp_device(c->mlp);
      lbm::ClosureEval e{};
      e.nb = 2 * (c->p.nx - 2) + (c->p.ny - 2);
      e.blocks = lbm::closure_blocks(e.nb);
      e.mask = c->closure_mask;
      e.taper = c->closure_taper;
      e.outlet_taper = c->closure_outlet_taper;
      e.outlet_neutral = c->closure_outlet_neutral;
      e.beta = c->closure_beta;
      e.limit = c->closure_limit;
      e.Wb = md.Wb;
      e.master = md.master;
      e.norm = c->d_norm;
      e.bias = c->d_bias;
      e.resid_in = c->d_resid[c->rc];
      e.resid = c->d_resid[c->rc ^ 1];
      if (lbm::step_fuses_closure(v, k))
        a.ev = e;
      else
        HIP_TRY(lbm::launch_closure(a.A, c->geo, e, s));
    }
    a.closure = c->d_resid[c->rc];
    a.closure_mask = c->closure_mask;
  }
  HIP_TRY(lbm::launch_step(a, v, s));
  c->cur ^= 1;
  c->step += k;
  c->pending += k;
  if (c->pending == lbm::kRing) {
    HIP_TRY(lbm::launch_force_reduce(c->d_partials, slots_of(c), c->pending, c->d_hist,
                                     c->p.hist_capacity, c->d_step, c->d_bad, c->d_bad_step, s));
    c->pending = 0;
  }
  return LBM_OK;
}

// Captures kRing steps starting from buf[c->cur] (ring empty) into a graph.
lbm_status capture(lbm_ctx* c) {
  if (!c->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
  const int cur0 = c->cur, rc0 = c->rc, gi = cur0 | (rc0 << 1);
  const int64_t step0 = c->step;
  HIP_TRY(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
  lbm_status st = LBM_OK;
  int launches = 0;
  for (int i = 0; i < lbm::kRing && st == LBM_OK; ++launches) {
    const int k = group(c, lbm::kRing - i);
    st = enqueue_step(c, c->capture_stream, k);
    i += k;
  }
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
  const int evals = c->rc != rc0;
  c->cur = cur0;  // capturing ran nothing
  c->step = step0;
  c->pending = 0;
  c->rc = rc0;
  if (st != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(LBM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  const hipError_t e2 = hipGraphInstantiate(&c->graph[gi], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return fail(LBM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  c->graph_flip[gi] = launches & 1;
  c->resid_flip[gi] = evals;
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_set_graphs(lbm_ctx* c, int enable) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  c->use_graphs = enable ? 1 : 0;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t steps, const char* cache_path, int32_t* best) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (steps < 1) return fail(LBM_ERR_INVALID_ARG, "steps must be >= 1");
  char key[128];
  snprintf(key, sizeof key, "lattice-%dx%d-d%d-w%d-x%d", c->p.nx, c->p.ny, c->p.diameter, c->p.wall,
           c->p.x_periodic);
  int v_best = 0;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char k[256];
      int v = 0;
      while (fscanf(f, "%255s %d", k, &v) == 2)
        if (!strcmp(k, key) && v >= 1 && v <= lbm::num_variants()) v_best = v;
      fclose(f);
    }
  }
  if (!v_best) {
    lbm_ctx* scratch = nullptr;
    lbm_status st = lbm_create(&c->p, c->stream, &scratch);
    if (st != LBM_OK) return st;
    scratch->use_graphs = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float t_best = 1e30f;
    st = LBM_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
      st = fail(LBM_ERR_HIP, "hipEventCreate failed");
    for (int v = 1; st == LBM_OK && v <= lbm::num_variants(); ++v) {
      if ((st = lbm_set_variant(scratch, v)) != LBM_OK) break;
      if ((st = lbm_step(scratch, 4)) != LBM_OK) break;
      (void)hipEventRecord(e0, scratch->stream);
      if ((st = lbm_step(scratch, steps)) != LBM_OK) break;
      (void)hipEventRecord(e1, scratch->stream);
      float ms = 1e30f;
      if (hipEventSynchronize(e1) == hipSuccess) (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < t_best) {
        t_best = ms;
        v_best = v;
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    lbm_destroy(scratch);
    if (st != LBM_OK) return st;
    if (cache_path)
      if (FILE* f = fopen(cache_path, "a")) {
        fprintf(f, "%s %d\n", key, v_best);
        fclose(f);
      }
  }
  lbm_status st = lbm_set_variant(c, v_best);
  if (st == LBM_OK && best) *best = v_best;
  return st;
}

lbm_status lbm_closure_enable(lbm_ctx* c, lbm_mlp* m, const float* norm, int32_t boundaries) {
  if (check_ctx(c) || !m || !norm) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  if (boundaries < 0 || boundaries > 7) return fail(LBM_ERR_INVALID_ARG, "boundary mask must be in 0..7");
  if (c->p.wall != LBM_WALL_FREE_SLIP || c->p.outlet_mode != LBM_OUTLET_COPY_UNKNOWN || c->p.x_periodic)
    return fail(LBM_ERR_INVALID_ARG, "the closure refines free-slip walls and the copy-unknown outlet");
  lbm_status st = flush(c);
  if (st != LBM_OK) return st;
  drop_graphs(c);
  const size_t nb = 2 * (size_t)(c->p.nx - 2) + (size_t)(c->p.ny - 2);
  if (!c->d_norm) HIP_TRY(hipMalloc(&c->d_norm, sizeof(float) * lbm::kClosureNorm));
  for (int i = 0; i < 2; ++i) {
    if (!c->d_resid[i]) HIP_TRY(hipMalloc(&c->d_resid[i], sizeof(float) * 3 * nb));
    HIP_TRY(hipMemsetAsync(c->d_resid[i], 0, sizeof(float) * 3 * nb, c->stream));
  }
  c->rc = 1;  // the first evaluation makes d_resid[0] (zeros) the one in use
  HIP_TRY(hipMemcpyAsync(c->d_norm, norm, sizeof(float) * lbm::kClosureNorm, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->mlp = m;
  c->closure_mask = boundaries;
  return LBM_OK;
}

lbm_status lbm_closure_set_filter(lbm_ctx* c, float beta, int32_t taper) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (!(beta > 0.0f && beta <= 1.0f)) return fail(LBM_ERR_INVALID_ARG, "beta must be in (0, 1]");
  if (taper < 0) return fail(LBM_ERR_INVALID_ARG, "taper must be >= 0");
  drop_graphs(c);
  c->closure_beta = beta;
  c->closure_taper = taper;
  return LBM_OK;
}

lbm_status lbm_closure_set_guard(lbm_ctx* c, float limit, int32_t outlet_taper, int32_t outlet_neutral) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (!(limit >= 0.0f)) return fail(LBM_ERR_INVALID_ARG, "limit must be >= 0");
  if (outlet_taper < 0) return fail(LBM_ERR_INVALID_ARG, "outlet_taper must be >= 0");
  drop_graphs(c);
  c->closure_limit = limit;
  c->closure_outlet_taper = outlet_taper;
  c->closure_outlet_neutral = outlet_neutral != 0;
  return LBM_OK;
}

lbm_status lbm_closure_set_bias(lbm_ctx* c, const float* bias) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  lbm_status st = flush(c);
  if (st != LBM_OK) return st;
  drop_graphs(c);
  if (!bias) {
    (void)hipFree(c->d_bias);
    c->d_bias = nullptr;
    return LBM_OK;
  }
  const size_t nb = 2 * (size_t)(c->p.nx - 2) + (size_t)(c->p.ny - 2);
  if (!c->d_bias) HIP_TRY(hipMalloc(&c->d_bias, sizeof(float) * 3 * nb));
  HIP_TRY(hipMemcpyAsync(c->d_bias, bias, sizeof(float) * 3 * nb, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_closure_set_interval(lbm_ctx* c, int32_t interval) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (interval < 1 || interval > lbm::kRing || lbm::kRing % interval != 0)
    return fail(LBM_ERR_INVALID_ARG, "interval %d must divide %d", interval, lbm::kRing);
  lbm_status st = flush(c);
  if (st != LBM_OK) return st;
  drop_graphs(c);
  c->closure_interval = interval;
  return LBM_OK;
}

lbm_status lbm_closure_disable(lbm_ctx* c) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  lbm_status st = flush(c);
  if (st != LBM_OK) return st;
  drop_graphs(c);
  c->mlp = nullptr;
  return LBM_OK;
}

lbm_status lbm_closure_residuals(lbm_ctx* c, float* out) {
  if (check_ctx(c) || !out) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  if (!c->mlp) return fail(LBM_ERR_STATE, "closure not enabled");
  const size_t nb = 2 * (size_t)(c->p.nx - 2) + (size_t)(c->p.ny - 2);
  const lbm::MlpDevice md = lbm::mlp_device(c->mlp);
  if (!c->d_resid_q) HIP_TRY(hipMalloc(&c->d_resid_q, sizeof(float) * 3 * nb));
  lbm::ClosureEval e{};
  e.nb = (int)nb;
  e.mask = c->closure_mask;
  e.taper = c->closure_taper;
  e.outlet_taper = c->closure_outlet_taper;
  e.outlet_neutral = c->closure_outlet_neutral;
  e.beta = 1.0f;
  e.limit = c->closure_limit;
  e.Wb = md.Wb;
  e.master = md.master;
  e.norm = c->d_norm;
  e.bias = c->d_bias;
  e.resid_in = c->d_resid_q;
  e.resid = c->d_resid_q;
  HIP_TRY(lbm::launch_closure(c->buf[c->cur], c->geo, e, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(out, c->d_resid_q, sizeof(float) * 3 * nb, hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_sample_boundary(lbm_ctx* c, int32_t ox, int32_t oy, int32_t wnx, int32_t wny,
                               const int32_t* nodes, int64_t n, const float* bias, float* feat, float* target) {
  if (check_ctx(c) || !nodes || !feat || !target || n < 0 || n > INT_MAX)
    return fail(LBM_ERR_INVALID_ARG, "bad sampling arguments");
  // the window, its two inward layers and the outside neighbours it pulls from
  if (wnx < 4 || wny < 4 || ox < 0 || oy < 1 || ox + wnx > c->p.nx - 1 || oy + wny > c->p.ny - 1)
    return fail(LBM_ERR_INVALID_ARG, "window %dx%d at (%d, %d) does not fit in the %dx%d lattice", wnx, wny, ox,
                oy, c->p.nx, c->p.ny);
  if (n == 0) return LBM_OK;
  lbm_status st = flush(c);
  if (st != LBM_OK) return st;
  HIP_TRY(lbm::launch_sample_boundary(c->buf[c->cur], c->geo, ox, oy, wnx, wny, nodes, (int)n, bias, feat,
                                      target, c->stream));
  return LBM_OK;
}

lbm_status lbm_copy_probe(void* dst, const void* src, int64_t nbytes, void* stream) {
  if (!dst || !src || nbytes < 0 || nbytes % 16) return fail(LBM_ERR_INVALID_ARG, "bad copy probe arguments");
  if (nbytes == 0) return LBM_OK;
  HIP_TRY(lbm::launch_copy_probe(dst, src, nbytes, (hipStream_t)stream));
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (n < 0) return fail(LBM_ERR_INVALID_ARG, "n must be >= 0");
  int64_t i = 0;
  // plain launches until the ring is empty (and, with a learned closure, the
  // step index is a multiple of its interval, so that every graph replays
  // the evaluations at the same places), then whole graphs
  while (i < n && (c->pending != 0 || (c->mlp && c->step % c->closure_interval != 0))) {
    const int k = group(c, n - i);
    lbm_status st = enqueue_step(c, c->stream, k);
    if (st != LBM_OK) return st;
    i += k;
  }
  if (c->use_graphs) {
    while (n - i >= lbm::kRing) {
      const int gi = c->cur | (c->rc << 1);
      if (!c->graph[gi]) {
        lbm_status st = capture(c);
        if (st != LBM_OK) return st;
      }
      HIP_TRY(hipGraphLaunch(c->graph[gi], c->stream));
      c->cur ^= c->graph_flip[gi];
      c->rc ^= c->resid_flip[gi];
      c->step += lbm::kRing;
      i += lbm::kRing;
    }
  }
  while (i < n) {
    const int k = group(c, n - i);
    lbm_status st = enqueue_step(c, c->stream, k);
    if (st != LBM_OK) return st;
    i += k;
  }
  return flush(c);
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  HIP_TRY(hipStreamSynchronize(c->stream));
  int64_t bad = 0;
  HIP_TRY(hipMemcpy(&bad, c->d_bad_step, sizeof bad, hipMemcpyDeviceToHost));
  if (bad) return fail(LBM_ERR_DIVERGED, "density left (0, 10) or became non-finite at step %lld", (long long)bad);
  return LBM_OK;
}

lbm_status lbm_get_step(lbm_ctx* c, int64_t* step) {
  if (check_ctx(c) || !step) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  *step = c->step;
  return LBM_OK;
}

lbm_status lbm_diverged_step(lbm_ctx* c, int64_t* step) {
  if (check_ctx(c) || !step) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(c->stream));
  HIP_TRY(hipMemcpy(step, c->d_bad_step, sizeof *step, hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_forces(lbm_ctx* c, int64_t first, int64_t count, double* fx, double* fy, double* cd,
                      double* cl) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  if (count < 0 || first < 1) return fail(LBM_ERR_INVALID_ARG, "first must be >= 1 and count >= 0");
  const int64_t cap = c->p.hist_capacity;
  if (first + count - 1 > c->step || first <= c->step - cap)
    return fail(LBM_ERR_RANGE, "steps [%lld, %lld] not stored (have (%lld, %lld])", (long long)first,
                (long long)(first + count - 1), (long long)std::max<int64_t>(0, c->step - cap),
                (long long)c->step);
  if ((cd || cl) && !(c->p.u_in > 0 && c->p.diameter > 0))
    return fail(LBM_ERR_INVALID_ARG, "coefficients need u_in > 0 and diameter > 0");
  lbm_status st = lbm_sync(c);
  if (st != LBM_OK && st != LBM_ERR_DIVERGED) return st;
  if (count == 0) return st;
  std::vector<double> h((size_t)2 * count);
  // the ring may wrap: copy in at most two pieces
  int64_t done = 0;
  while (done < count) {
    const int64_t s = (first - 1 + done) % cap;
    const int64_t n = std::min(count - done, cap - s);
    HIP_TRY(hipMemcpy(h.data() + 2 * done, c->d_hist + 2 * s, sizeof(double) * 2 * n, hipMemcpyDeviceToHost));
    done += n;
  }
  const double q = 0.5 * 1.0 * c->p.u_in * c->p.u_in * c->p.diameter;  // Eq. 15, rho_in = 1
  for (int64_t i = 0; i < count; ++i) {
    if (fx) fx[i] = h[2 * i];
    if (fy) fy[i] = h[2 * i + 1];
    if (cd) cd[i] = h[2 * i] / q;
    if (cl) cl[i] = h[2 * i + 1] / q;
  }
  return st;
}

lbm_status lbm_fields(lbm_ctx* c, float* rho, float* ux, float* uy, int on_device) {
  if (check_ctx(c)) return LBM_ERR_INVALID_ARG;
  const lbm::Geometry& g = c->geo;
  const size_t n = (size_t)g.nx * g.ny;
  if (on_device) {
    HIP_TRY(lbm::launch_fields(c->buf[c->cur], g, rho, ux, uy, c->stream));
    return lbm_sync(c);
  }
  float* d = nullptr;
  HIP_TRY(hipMalloc(&d, 3 * n * sizeof(float)));
  lbm_status st = LBM_OK;
  hipError_t e = lbm::launch_fields(c->buf[c->cur], g, d, d + n, d + 2 * n, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && rho) e = hipMemcpy(rho, d, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && ux) e = hipMemcpy(ux, d + n, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess && uy) e = hipMemcpy(uy, d + 2 * n, n * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) st = fail(LBM_ERR_HIP, "lbm_fields: %s", hipGetErrorString(e));
  (void)hipFree(d);
  if (st != LBM_OK) return st;
  return lbm_sync(c);
}

lbm_status lbm_get_populations(lbm_ctx* c, void* buf, int dtype, int on_device) {
  if (check_ctx(c) || !buf) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  if (dtype != 0 && dtype != 1) return fail(LBM_ERR_INVALID_ARG, "dtype must be 0 (f32) or 1 (f64)");
  const lbm::Geometry& g = c->geo;
  const size_t bytes = (size_t)9 * g.nx * g.ny * (dtype ? 8 : 4);
  if (on_device) {
    HIP_TRY(lbm::launch_pack(c->buf[c->cur], g, buf, dtype, c->stream));
    return lbm_sync(c);
  }
  void* d = nullptr;
  HIP_TRY(hipMalloc(&d, bytes));
  hipError_t e = lbm::launch_pack(c->buf[c->cur], g, d, dtype, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(buf, d, bytes, hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_ERR_HIP, "lbm_get_populations: %s", hipGetErrorString(e));
  return lbm_sync(c);
}

lbm_status lbm_set_populations(lbm_ctx* c, const void* buf, int dtype, int on_device) {
  if (check_ctx(c) || !buf) return fail(LBM_ERR_INVALID_ARG, "NULL argument");
  if (dtype != 0 && dtype != 1) return fail(LBM_ERR_INVALID_ARG, "dtype must be 0 (f32) or 1 (f64)");
  const lbm::Geometry& g = c->geo;
  const size_t bytes = (size_t)9 * g.nx * g.ny * (dtype ? 8 : 4);
  if (on_device) {
    HIP_TRY(lbm::launch_unpack(buf, dtype, g, c->buf[c->cur], c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
  }
  void* d = nullptr;
  HIP_TRY(hipMalloc(&d, bytes));
  hipError_t e = hipMemcpyAsync(d, buf, bytes, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = lbm::launch_unpack(d, dtype, g, c->buf[c->cur], c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_ERR_HIP, "lbm_set_populations: %s", hipGetErrorString(e));
  return LBM_OK;
}

// ------------------------------------------------------------------ statistics
lbm_status lbm_shedding_stats(const double* cd, const double* cl, int64_t n, double d, double u,
                              int32_t periods, lbm_shedding* out) {
  if (!cd || !cl || !out || n < 2 || periods < 1 || !(u > 0) || !(d > 0))
    return fail(LBM_ERR_INVALID_ARG, "bad arguments to lbm_shedding_stats");
  auto crossings = [&](double level, std::vector<double>& xs) {
    xs.clear();
    for (int64_t i = 0; i + 1 < n; ++i) {
      const double a = cl[i] - level, b = cl[i + 1] - level;
      if (a < 0.0 && b >= 0.0) xs.push_back((double)i + (-a) / (b - a));
    }
  };
  double mean = 0.0;
  for (int64_t i = 0; i < n; ++i) mean += cl[i];
  mean /= (double)n;
  std::vector<double> xs;
  crossings(mean, xs);
  if ((int64_t)xs.size() < periods + 1) return fail(LBM_ERR_RANGE, "only %zu lift crossings", xs.size());
  double a0 = xs[xs.size() - periods - 1], a1 = xs.back();
  double T = (a1 - a0) / periods;
  int64_t i0 = (int64_t)std::ceil(a0), i1 = (int64_t)std::floor(a1);
  // second pass about the window's own mean
  double wm = 0.0;
  for (int64_t i = i0; i <= i1; ++i) wm += cl[i];
  wm /= (double)(i1 - i0 + 1);
  std::vector<double> ys;
  crossings(wm, ys);
  std::vector<double> keep;
  for (double v : ys)
    if (v >= a0 - 0.5 * T) keep.push_back(v);
  if ((int64_t)keep.size() >= periods + 1) {
    a0 = keep[keep.size() - periods - 1];
    a1 = keep.back();
    T = (a1 - a0) / periods;
    i0 = (int64_t)std::ceil(a0);
    i1 = (int64_t)std::floor(a1);
  }
  double lo = INFINITY, hi = -INFINITY, sd = 0.0;
  for (int64_t i = i0; i <= i1; ++i) {
    lo = std::min(lo, cl[i]);
    hi = std::max(hi, cl[i]);
    sd += cd[i];
  }
  out->mean_cd = sd / (double)(i1 - i0 + 1);
  out->cl_amp = 0.5 * (hi - lo);
  out->st = d / (T * u);
  out->period = T;
  return LBM_OK;
}

}  // extern "C"
