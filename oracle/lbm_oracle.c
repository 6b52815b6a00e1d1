/*
 * FP64 CPU oracle for the D2Q9 BGK cylinder-flow method (arXiv 2605.02185).
 * TEST INFRASTRUCTURE ONLY: see lbm_oracle.h.  Built with gcc; never linked
 * into the GPU library.
 *
 * One time step, in the paper's order (Sec. 2.1, last paragraph):
 *   O1 collide every fluid node (Eqs. 2-4)
 *   O2 momentum-exchange force from the post-collision populations (Eq. 14)
 *   O3 push-stream; a population that would enter a solid node is flipped
 *      back into the opposite direction of its own node in the same step
 *      (half-way bounce-back, Sec. 3.1)
 *   O4 top and bottom rows (Sec. 2.3.1-2.3.4)
 *   O5 outlet column, zeroth-order extrapolation (Eq. 13)
 *   O6 velocity inlet column, Zou-He (Sec. 3.1)
 *   O7 inlet corners
 *   O8 the corrected populations become the new state
 * Targets that nothing writes in O3 are the populations missing at the domain
 * edges (Fig. 2); they are set to NaN before streaming so that a boundary pass
 * that forgets one is caught by the finiteness check below.
 *
 * Every pass is pinned by a test against the paper or the mathematics
 * (tests/test_oracle_*.py).
 */
#include "lbm_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Table 1 with k = i - 1. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W[9] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* opposite direction: c_opp(k) = -c_k */
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

enum { R = 0, E = 1, N = 2, Wd = 3, S = 4, NE = 5, NW = 6, SW = 7, SE = 8 };

/* Eq. 6: the transformation matrix M to the moments
 * (rho, e, epsilon, j_x, q_x, j_y, q_y, p_xx, p_xy), columns in Table 1 order. */
static const double MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},          {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},      {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},       {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},       {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

void oracle_mrt_matrix(double* M) {
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) M[i * 9 + j] = MRT_M[i][j];
}

/* The equilibrium moments of Sec. 2.1, read with the factor rho that makes
 * them the moments of the equilibrium of Eq. 3 (the printed list omits it). */
void oracle_mrt_meq(double rho, double ux, double uy, double* m) {
  double uu = ux * ux + uy * uy;
  m[0] = rho;
  m[1] = rho * (-2.0 + 3.0 * uu);
  m[2] = rho * (1.0 - 3.0 * uu);
  m[3] = rho * ux;
  m[4] = -rho * ux;
  m[5] = rho * uy;
  m[6] = -rho * uy;
  m[7] = rho * (ux * ux - uy * uy);
  m[8] = rho * ux * uy;
}

/* M^{-1} by Gauss-Jordan elimination with partial pivoting (once). */
static double MRT_MINV[9][9];
static int mrt_ready = 0;
static void mrt_invert(void) {
  double a[9][18];
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 18; ++j) a[i][j] = j < 9 ? MRT_M[i][j] : (j - 9 == i ? 1.0 : 0.0);
  for (int c = 0; c < 9; ++c) {
    int piv = c;
    for (int r = c + 1; r < 9; ++r)
      if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
    for (int j = 0; j < 18; ++j) {
      double t = a[c][j];
      a[c][j] = a[piv][j];
      a[piv][j] = t;
    }
    double d = a[c][c];
    for (int j = 0; j < 18; ++j) a[c][j] /= d;
    for (int r = 0; r < 9; ++r) {
      if (r == c) continue;
      double f = a[r][c];
      for (int j = 0; j < 18; ++j) a[r][j] -= f * a[c][j];
    }
  }
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) MRT_MINV[i][j] = a[i][j + 9];
  mrt_ready = 1;
}

struct oracle {
  oracle_params p;
  int nx, ny;
  double tau;
  double u_top, u_bot;
  unsigned char* solid; /* [ny][nx] */
  double* f;            /* state f(t), [ny][nx][9] */
  double* fs;           /* post-collision f*(t) */
  double* g;            /* streamed populations f(t+1) under construction */
  double* rho_t;        /* density of f(t) per node, used by Eq. 11 */
  int state_is_post;    /* 1: f holds f*(t) (set by oracle_set_fstar) */
  long t;
  double s[9];          /* MRT relaxation rates */
  /* fluid-to-solid links (node, direction) in row-major node order, fixed at
   * creation; the force sum of Eq. 14 runs over them in this order */
  long n_links;
  size_t* link_node;
  int* link_dir;
  double* link_q;       /* wall fraction of each link (interpolated bounce-back) */
  double* node_q;       /* [ny][nx][9]: q of the link (node, k), NaN elsewhere */
  int own_mask;         /* the caller supplied the solid mask */
};

static size_t node(const oracle* o, int x, int y) { return (size_t)y * o->nx + x; }

/* Eq. 3 with c = 1: f_eq_k = w_k rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u] */
static double feq(int k, double rho, double ux, double uy) {
  double cu = CX[k] * ux + CY[k] * uy;
  double uu = ux * ux + uy * uy;
  return W[k] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

double oracle_tau(const oracle_params* p) {
  if (p->tau > 0) return p->tau;
  double nu = p->u_in * p->diameter / p->re; /* Eq. 16 */
  return 3.0 * nu + 0.5;                     /* Eq. 17 */
}

long oracle_digitise(const oracle_params* p, unsigned char* solid) {
  long count = 0;
  long d2 = (long)p->diameter * p->diameter;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x) {
      long dx = 2L * x - p->cx2, dy = 2L * y - p->cy2;
      int s = p->diameter > 0 && dx * dx + dy * dy <= d2;
      solid[(size_t)y * p->nx + x] = (unsigned char)s;
      count += s;
    }
  return count;
}

/* With full-way bounce-back the solid nodes carry populations; they start
 * at rest, f = w (which their reversal leaves unchanged). */
static void init_equilibrium(oracle* o) {
  const double U = o->p.u_in, a = o->p.perturb_amp;
  const double pi = 3.14159265358979323846;
  for (int y = 0; y < o->ny; ++y) {
    double v = o->ny > 1 ? a * U * sin(2.0 * pi * y / (o->ny - 1)) : 0.0;
    for (int x = 0; x < o->nx; ++x) {
      size_t n = node(o, x, y);
      int rest = o->p.bounce == ORACLE_BB_FULLWAY && o->solid[n];
      for (int k = 0; k < 9; ++k) o->f[n * 9 + k] = rest ? W[k] : feq(k, 1.0, U, v);
    }
  }
}

static int build_links(oracle* o);

oracle* oracle_create(const oracle_params* p, const unsigned char* solid) {
  if (!p || p->nx < 3 || p->ny < 3) return NULL;
  /* the body force is a BGK-only test device (Guo forcing in the BGK form) */
  if (p->collision == ORACLE_MRT && (p->gx != 0.0 || p->gy != 0.0)) return NULL;
  oracle* o = (oracle*)calloc(1, sizeof(oracle));
  if (!o) return NULL;
  o->p = *p;
  o->nx = p->nx;
  o->ny = p->ny;
  o->tau = oracle_tau(p);
  o->u_top = isnan(p->u_wall_top) ? p->u_in : p->u_wall_top;
  o->u_bot = isnan(p->u_wall_bottom) ? p->u_in : p->u_wall_bottom;
  for (int i = 0; i < 9; ++i) o->s[i] = p->s_rates[i];
  if (!(o->s[7] > 0)) o->s[7] = 1.0 / o->tau;
  if (!(o->s[8] > 0)) o->s[8] = 1.0 / o->tau;
  if (!mrt_ready) mrt_invert();
  size_t nn = (size_t)o->nx * o->ny;
  o->solid = (unsigned char*)malloc(nn);
  o->f = (double*)malloc(nn * 9 * sizeof(double));
  o->fs = (double*)malloc(nn * 9 * sizeof(double));
  o->g = (double*)malloc(nn * 9 * sizeof(double));
  o->rho_t = (double*)malloc(nn * sizeof(double));
  if (!o->solid || !o->f || !o->fs || !o->g || !o->rho_t) {
    oracle_destroy(o);
    return NULL;
  }
  if (solid)
    memcpy(o->solid, solid, nn);
  else
    oracle_digitise(p, o->solid);
  init_equilibrium(o);
  o->own_mask = solid != NULL;
  if (build_links(o) != 0) {
    oracle_destroy(o);
    return NULL;
  }
  return o;
}

void oracle_destroy(oracle* o) {
  if (!o) return;
  free(o->solid);
  free(o->f);
  free(o->fs);
  free(o->g);
  free(o->rho_t);
  free(o->link_node);
  free(o->link_dir);
  free(o->link_q);
  free(o->node_q);
  free(o);
}

long oracle_time(const oracle* o) { return o->t; }

/* Moments of Eq. 4 at one node; with a body force the velocity is shifted by
 * half the force (Guo et al. 2002), which only the test boxes use. */
static void moments(const oracle* o, const double* fn, double* rho, double* ux, double* uy) {
  double r = 0, mx = 0, my = 0;
  for (int k = 0; k < 9; ++k) {
    r += fn[k];
    mx += CX[k] * fn[k];
    my += CY[k] * fn[k];
  }
  *rho = r;
  *ux = (mx + 0.5 * r * o->p.gx) / r;
  *uy = (my + 0.5 * r * o->p.gy) / r;
}

/* O1: BGK collision f* = f - (f - f_eq)/tau (Eq. 2).  Returns 1 if some fluid
 * density is non-finite or outside (0, 10). */
static int collide(oracle* o) {
  int bad = 0;
  const double tau = o->tau;
  const int forced = o->p.gx != 0.0 || o->p.gy != 0.0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int y = 0; y < o->ny; ++y) {
    for (int x = 0; x < o->nx; ++x) {
      size_t n = node(o, x, y);
      const double* fn = o->f + n * 9;
      double* out = o->fs + n * 9;
      if (o->solid[n]) {
        /* full-way bounce-back: the populations that arrived are sent back
         * (a state given as post-collision is already reversed) */
        int reverse = o->p.bounce == ORACLE_BB_FULLWAY && !o->state_is_post;
        for (int k = 0; k < 9; ++k) out[k] = reverse ? fn[OPP[k]] : fn[k];
        o->rho_t[n] = 1.0;
        continue;
      }
      double rho, ux, uy;
      moments(o, fn, &rho, &ux, &uy);
      o->rho_t[n] = rho;
      if (!(rho > 0.0 && rho < 10.0)) bad = 1;
      if (o->state_is_post) {
        for (int k = 0; k < 9; ++k) out[k] = fn[k];
        continue;
      }
      if (o->p.collision == ORACLE_MRT) {
        /* Eq. 6: f* = f - M^{-1} S M (f - f_eq), with M f_eq = m_eq */
        double m[9], meq[9], dm[9];
        for (int i = 0; i < 9; ++i) {
          m[i] = 0.0;
          for (int k = 0; k < 9; ++k) m[i] += MRT_M[i][k] * fn[k];
        }
        oracle_mrt_meq(rho, ux, uy, meq);
        for (int i = 0; i < 9; ++i) dm[i] = o->s[i] * (m[i] - meq[i]);
        for (int k = 0; k < 9; ++k) {
          double acc = 0.0;
          for (int i = 0; i < 9; ++i) acc += MRT_MINV[k][i] * dm[i];
          out[k] = fn[k] - acc;
        }
        continue;
      }
      for (int k = 0; k < 9; ++k) {
        double fk = fn[k];
        out[k] = fk - (fk - feq(k, rho, ux, uy)) / tau;
        if (forced) {
          /* Guo source term, test boxes only */
          double cu = CX[k] * ux + CY[k] * uy;
          double fx = rho * o->p.gx, fy = rho * o->p.gy;
          double src = W[k] * (3.0 * ((CX[k] - ux) * fx + (CY[k] - uy) * fy) + 9.0 * cu * (CX[k] * fx + CY[k] * fy));
          out[k] += (1.0 - 0.5 / tau) * src;
        }
      }
    }
  }
  o->state_is_post = 0;
  return bad;
}

/* Neighbour of (x, y) along c_k.  Wraps in y for periodic walls and in x for
 * periodic test boxes.  Returns 0 if it falls outside the lattice. */
static int neighbour(const oracle* o, int x, int y, int k, int* xo, int* yo) {
  int xn = x + CX[k], yn = y + CY[k];
  if (o->p.x_periodic) xn = (xn + o->nx) % o->nx;
  if (o->p.wall == ORACLE_WALL_PERIODIC) yn = (yn + o->ny) % o->ny;
  if (xn < 0 || xn >= o->nx || yn < 0 || yn >= o->ny) return 0;
  *xo = xn;
  *yo = yn;
  return 1;
}

/* Sec. 2.4 (link-wise approach, Bouzidi, Firdaouss & Lallemand 2001): the
 * wall cuts the link from the fluid node x along c_k at x + q c_k.  For the
 * cylinder, the circle |p - c| = D/2 with c = (cx2, cy2)/2; in doubled
 * coordinates X = 2x - cx2, Y = 2y - cy2 the cut solves
 * (X + 2 q cx)^2 + (Y + 2 q cy)^2 = D^2, whose smaller root lies in (0, 1]
 * because x is outside the digitised disk and x + c_k inside or on it. */
static double link_fraction(const oracle* o, int x, int y, int k) {
  if (o->p.q_fixed > 0.0) return o->p.q_fixed;
  if (o->own_mask || o->p.diameter <= 0) return 0.5;
  double X = 2.0 * x - o->p.cx2, Y = 2.0 * y - o->p.cy2, D = o->p.diameter;
  double a = 4.0 * (CX[k] * CX[k] + CY[k] * CY[k]);
  double b = 4.0 * (X * CX[k] + Y * CY[k]);
  double c = X * X + Y * Y - D * D;
  double disc = b * b - 4.0 * a * c;
  if (disc < 0.0) disc = 0.0;
  double q = (-b - sqrt(disc)) / (2.0 * a);
  if (q <= 0.0) q = 1e-12;
  if (q > 1.0) q = 1.0;
  return q;
}

/* Every link from a fluid node into a solid node, all eight directions, in
 * row-major node order. */
static int build_links(oracle* o) {
  long cap = 0, n = 0;
  for (int pass = 0; pass < 2; ++pass) {
    n = 0;
    for (int y = 0; y < o->ny; ++y)
      for (int x = 0; x < o->nx; ++x) {
        size_t m = node(o, x, y);
        if (o->solid[m]) continue;
        for (int k = 1; k < 9; ++k) {
          int xn, yn;
          if (!neighbour(o, x, y, k, &xn, &yn) || !o->solid[node(o, xn, yn)]) continue;
          if (pass == 1) {
            o->link_node[n] = m;
            o->link_dir[n] = k;
            o->link_q[n] = link_fraction(o, x, y, k);
            if (o->node_q) o->node_q[m * 9 + k] = o->link_q[n];
          }
          ++n;
        }
      }
    if (pass == 0) {
      cap = n > 0 ? n : 1;
      o->link_node = (size_t*)malloc(cap * sizeof(size_t));
      o->link_dir = (int*)malloc(cap * sizeof(int));
      o->link_q = (double*)malloc(cap * sizeof(double));
      if (!o->link_node || !o->link_dir || !o->link_q) return -1;
      if (o->p.bounce == ORACLE_BB_INTERP) {
        size_t nn9 = (size_t)o->nx * o->ny * 9;
        o->node_q = (double*)malloc(nn9 * sizeof(double));
        if (!o->node_q) return -1;
        for (size_t i = 0; i < nn9; ++i) o->node_q[i] = NAN;
      }
    }
  }
  o->n_links = n;
  return 0;
}

long oracle_links(const oracle* o, long* out_node, int* out_dir, double* out_q) {
  for (long i = 0; i < o->n_links; ++i) {
    if (out_node) out_node[i] = (long)o->link_node[i];
    if (out_dir) out_dir[i] = o->link_dir[i];
    if (out_q) out_q[i] = o->link_q[i];
  }
  return o->n_links;
}

/* The population that comes back to fluid node n along -c_k after its
 * post-collision f*_k(n) has met the wall of link (n, k) with fraction q.
 * Half-way bounce-back: f*_k(n).  Interpolated (the linear scheme of Bouzidi
 * et al.): for q < 1/2 the value is interpolated between n and the fluid node
 * n - c_k behind it, 2 q f*_k(n) + (1 - 2q) f*_k(n - c_k); for q >= 1/2
 * between the reflected value and the node's own opposite population,
 * f*_k(n)/(2q) + (2q - 1)/(2q) f*_opp(k)(n).  Both give f*_k(n) at q = 1/2.
 * Where n - c_k is not a fluid node of the lattice, half-way bounce-back. */
static double bounced(const oracle* o, int x, int y, int k, double q) {
  size_t n = node(o, x, y);
  double fk = o->fs[n * 9 + k];
  if (o->p.bounce != ORACLE_BB_INTERP) return fk;
  if (q < 0.5) {
    int xb, yb;
    if (!neighbour(o, x, y, OPP[k], &xb, &yb) || o->solid[node(o, xb, yb)]) return fk;
    return 2.0 * q * fk + (1.0 - 2.0 * q) * o->fs[node(o, xb, yb) * 9 + k];
  }
  return fk / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * o->fs[n * 9 + OPP[k]];
}

/* O2: Eq. 14 summed over the links: the population leaving along c_k is
 * f*_k (in), the one coming back along -c_k is the bounced value (out), and
 * the body receives (f_in + f_out) c_k.  With half-way bounce-back both are
 * f*_k (stationary wall, same step): 2 c_k f*_k.  With full-way bounce-back
 * f*_k reaches the solid node in this step and leaves it reversed in the
 * next: the same 2 c_k f*_k, booked at this step. */
static void force(const oracle* o, double* fx, double* fy) {
  double sx = 0.0, sy = 0.0;
  for (long i = 0; i < o->n_links; ++i) {
    int k = o->link_dir[i];
    double f = o->fs[o->link_node[i] * 9 + k];
    if (o->p.bounce == ORACLE_BB_INTERP) {
      int x = (int)(o->link_node[i] % o->nx), y = (int)(o->link_node[i] / o->nx);
      double b = bounced(o, x, y, k, o->link_q[i]);
      sx += CX[k] * (f + b);
      sy += CY[k] * (f + b);
      continue;
    }
    sx += 2.0 * CX[k] * f;
    sy += 2.0 * CY[k] * f;
  }
  *fx = sx;
  *fy = sy;
}

/* O3: push streaming with bounce-back (half-way or interpolated) at solid
 * nodes; with full-way bounce-back (Sec. 3.1) solid nodes take part in the
 * streaming like fluid ones and reverse what arrived in their collision, so
 * a population that reaches the wall returns to its fluid node one step
 * later. */
static void stream(oracle* o) {
  long total = (long)o->nx * o->ny * 9;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < total; ++i) o->g[i] = NAN;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < o->ny; ++y)
    for (int x = 0; x < o->nx; ++x) {
      size_t n = node(o, x, y);
      int full = o->p.bounce == ORACLE_BB_FULLWAY;
      if (o->solid[n] && !full) continue;
      for (int k = 0; k < 9; ++k) {
        int xn, yn;
        if (!neighbour(o, x, y, k, &xn, &yn)) continue; /* leaves the lattice */
        size_t m = node(o, xn, yn);
        if (o->solid[m] && !full)
          o->g[n * 9 + OPP[k]] = o->node_q ? bounced(o, x, y, k, o->node_q[n * 9 + k]) : o->fs[n * 9 + k];
        else
          o->g[m * 9 + k] = o->fs[n * 9 + k];
      }
    }
}

/* O4: the top row (y = ny-1) is missing S, SW, SE; the bottom row (y = 0) is
 * missing N, NE, NW (Fig. 2). */
static void walls(oracle* o) {
  if (o->p.wall == ORACLE_WALL_PERIODIC) return;
  int x0 = o->p.x_periodic ? 0 : 1;
  int x1 = o->p.x_periodic ? o->nx - 1 : o->nx - 2;
  for (int x = x0; x <= x1; ++x) {
    for (int top = 0; top <= 1; ++top) {
      int y = top ? o->ny - 1 : 0;
      size_t n = node(o, x, y);
      if (o->solid[n]) continue;
      double* g = o->g + n * 9;
      const double* fs = o->fs + n * 9;
      double U = top ? o->u_top : o->u_bot;
      switch (o->p.wall) {
        case ORACLE_WALL_FREE_SLIP: /* Eq. 7: specular reflection */
          if (top) {
            g[S] = g[N];
            g[SW] = g[NW];
            g[SE] = g[NE];
          } else {
            g[N] = g[S];
            g[NW] = g[SW];
            g[NE] = g[SE];
          }
          break;
        case ORACLE_WALL_NEBB: { /* Eqs. 9-10, density from the known populations */
          if (top) {
            double rw = g[R] + g[E] + g[Wd] + 2.0 * (g[N] + g[NE] + g[NW]);
            g[S] = g[N];
            g[SW] = g[NE] + 0.5 * (g[E] - g[Wd]) - 0.5 * rw * U;
            g[SE] = g[NW] - 0.5 * (g[E] - g[Wd]) + 0.5 * rw * U;
          } else {
            double rw = g[R] + g[E] + g[Wd] + 2.0 * (g[S] + g[SW] + g[SE]);
            g[N] = g[S];
            g[NE] = g[SW] - 0.5 * (g[E] - g[Wd]) + 0.5 * rw * U;
            g[NW] = g[SE] + 0.5 * (g[E] - g[Wd]) - 0.5 * rw * U;
          }
          break;
        }
        case ORACLE_WALL_MOVING_BB: { /* Eq. 11: f_opp(i) = f*_i - 2 w_i rho (c_i.u_w)/cs^2 */
          double rho = o->rho_t[n];
          const int out_top[3] = {N, NE, NW};
          const int out_bot[3] = {S, SW, SE};
          const int* outk = top ? out_top : out_bot;
          for (int j = 0; j < 3; ++j) {
            int k = outk[j];
            g[OPP[k]] = fs[k] - 2.0 * W[k] * rho * (CX[k] * U) * 3.0;
          }
          break;
        }
        default:
          break;
      }
    }
  }
}

/* O5: zeroth-order extrapolation of the outlet column (Eq. 13).  Copy-all
 * takes all nine populations of x = nx - 2; copy-unknown only the ones no
 * streaming filled (Fig. 2): those whose source x - c_k lies outside the
 * lattice, i.e. c_kx = -1 and, at the two corners, the ones from beyond the
 * wall row. */
static void outlet(oracle* o) {
  if (o->p.x_periodic) return;
  int xo = o->nx - 1, xi = o->nx - 2;
  int yper = o->p.wall == ORACLE_WALL_PERIODIC;
  for (int y = 0; y < o->ny; ++y) {
    double* go = o->g + node(o, xo, y) * 9;
    const double* gi = o->g + node(o, xi, y) * 9;
    for (int k = 0; k < 9; ++k) {
      int sy = y - CY[k];
      int outside = xo - CX[k] >= o->nx || (!yper && (sy < 0 || sy >= o->ny));
      if (o->p.outlet_mode == ORACLE_OUTLET_COPY_ALL || outside) go[k] = gi[k];
    }
  }
}

/* O6: Zou-He velocity inlet with u = (U, 0).  The unknowns E, NE, SE follow
 * from the three moment equations of Eq. 4 plus bounce-back of the
 * non-equilibrium part normal to the inlet. */
static void inlet(oracle* o) {
  if (o->p.x_periodic) return;
  double U = o->p.u_in;
  int periodic = o->p.wall == ORACLE_WALL_PERIODIC;
  int y0 = periodic ? 0 : 1, y1 = periodic ? o->ny - 1 : o->ny - 2;
  for (int y = y0; y <= y1; ++y) {
    double* g = o->g + node(o, 0, y) * 9;
    double rho = (g[R] + g[N] + g[S] + 2.0 * (g[Wd] + g[NW] + g[SW])) / (1.0 - U);
    g[E] = g[Wd] + (2.0 / 3.0) * rho * U;
    g[NE] = g[SW] - 0.5 * (g[N] - g[S]) + rho * U / 6.0;
    g[SE] = g[NW] + 0.5 * (g[N] - g[S]) + rho * U / 6.0;
  }
  if (!periodic) { /* O7: inlet corners are Dirichlet equilibrium nodes */
    int ys[2] = {0, o->ny - 1};
    for (int j = 0; j < 2; ++j) {
      double* g = o->g + node(o, 0, ys[j]) * 9;
      for (int k = 0; k < 9; ++k) g[k] = feq(k, 1.0, U, 0.0);
    }
  }
}

long oracle_step(oracle* o, long nsteps, double* fx, double* fy) {
  for (long s = 0; s < nsteps; ++s) {
    int bad = collide(o);
    double Fx, Fy;
    force(o, &Fx, &Fy);
    if (fx) fx[s] = Fx;
    if (fy) fy[s] = Fy;
    stream(o);
    walls(o);
    outlet(o);
    inlet(o);
    /* O8 */
    long nn = (long)o->nx * o->ny;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long n = 0; n < nn; ++n) {
      if (o->solid[n] && o->p.bounce != ORACLE_BB_FULLWAY) continue;
      for (int k = 0; k < 9; ++k) {
        double v = o->g[n * 9 + k];
        if (!isfinite(v)) bad = 1;
        o->f[n * 9 + k] = v;
      }
    }
    o->t += 1;
    if (bad) return s + 1;
  }
  return 0;
}

void oracle_fields(const oracle* o, double* rho, double* ux, double* uy) {
  size_t nn = (size_t)o->nx * o->ny;
  for (size_t n = 0; n < nn; ++n) {
    if (o->solid[n]) {
      rho[n] = 1.0;
      ux[n] = 0.0;
      uy[n] = 0.0;
      continue;
    }
    moments(o, o->f + n * 9, rho + n, ux + n, uy + n);
  }
}

void oracle_get_f(const oracle* o, double* out) {
  size_t nn = (size_t)o->nx * o->ny;
  for (size_t n = 0; n < nn; ++n)
    for (int k = 0; k < 9; ++k) out[k * nn + n] = o->f[n * 9 + k];
}

void oracle_set_f(oracle* o, const double* in) {
  size_t nn = (size_t)o->nx * o->ny;
  for (size_t n = 0; n < nn; ++n)
    for (int k = 0; k < 9; ++k) o->f[n * 9 + k] = in[k * nn + n];
  o->state_is_post = 0;
}

void oracle_get_fstar(const oracle* o, double* out) {
  /* run the collision on a copy so the state is not advanced */
  oracle tmp = *o;
  size_t nn = (size_t)o->nx * o->ny;
  tmp.fs = (double*)malloc(nn * 9 * sizeof(double));
  tmp.rho_t = (double*)malloc(nn * sizeof(double));
  if (!tmp.fs || !tmp.rho_t) {
    free(tmp.fs);
    free(tmp.rho_t);
    for (size_t i = 0; i < nn * 9; ++i) out[i] = NAN;
    return;
  }
  collide(&tmp);
  for (size_t n = 0; n < nn; ++n)
    for (int k = 0; k < 9; ++k) out[k * nn + n] = tmp.fs[n * 9 + k];
  free(tmp.fs);
  free(tmp.rho_t);
}

void oracle_set_fstar(oracle* o, const double* in) {
  oracle_set_f(o, in);
  o->state_is_post = 1;
}

int oracle_threads(void) { return omp_get_max_threads(); }

/* Threads of the parallel loops that follow (n >= 1); timing only. */
void oracle_set_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
}
