/*
 * FP64 CPU oracle for the D2Q9 BGK lattice Boltzmann solver of unconfined flow
 * past a circular cylinder (Sahiti, Gurugubelli & Surasani, "Lattice Boltzmann
 * methodology for unconfined flows", arXiv 2605.02185).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never calls it, and it shares no code, header, table or helper with the GPU
 * path.
 *
 * The oracle is written for obviousness, not speed: array-of-structures state
 * f[y][x][k], push streaming into a fresh buffer, and each boundary treatment
 * as its own pass, in the order the paper gives (collide, stream, then the
 * boundary corrections; Sec. 2.1 and Sec. 2.3).
 *
 * Direction numbering k = 0..8 is the paper's Table 1 index i minus one:
 *   k : 0   1   2   3   4   5   6   7   8
 *   cx: 0   1   0  -1   0   1  -1  -1   1
 *   cy: 0   0   1   0  -1   1   1  -1  -1
 *   (rest, E, N, W, S, NE, NW, SW, SE)
 */
#ifndef LBM_ORACLE_H
#define LBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORACLE_WALL_FREE_SLIP = 0, /* Eq. 7 */
  ORACLE_WALL_PERIODIC = 1,  /* Eq. 8, read as wrap-around streaming in y */
  ORACLE_WALL_NEBB = 2,      /* Eqs. 9-10, wet-node Zou-He wall, u = (U_w, 0) */
  ORACLE_WALL_MOVING_BB = 3  /* Eq. 11, moving-wall bounce-back, u_w = (U_w, 0) */
};

enum { ORACLE_OUTLET_COPY_ALL = 0, ORACLE_OUTLET_COPY_UNKNOWN = 1 };

enum { ORACLE_BGK = 0, ORACLE_MRT = 1 };

enum { ORACLE_BB_HALFWAY = 0, ORACLE_BB_INTERP = 1, ORACLE_BB_FULLWAY = 2 };

typedef struct {
  int nx, ny;             /* lattice nodes x in [0,nx), y in [0,ny) */
  int diameter;           /* cylinder diameter in lattice units; 0 = no cylinder */
  int cx2, cy2;           /* cylinder centre in doubled coordinates (2*x_c, 2*y_c) */
  double u_in;            /* inlet velocity U */
  double re;              /* Reynolds number (used when tau <= 0) */
  double tau;             /* relaxation time; <= 0 derives it from Eqs. 16-17 */
  int wall;               /* ORACLE_WALL_* for the top and bottom rows */
  double u_wall_top;      /* tangential wall velocity, NaN = u_in */
  double u_wall_bottom;   /* tangential wall velocity, NaN = u_in */
  int outlet_mode;        /* ORACLE_OUTLET_* */
  int x_periodic;         /* 1 = periodic in x, no inlet/outlet (test boxes) */
  double perturb_amp;     /* initial v = amp*U*sin(2 pi y/(ny-1)) */
  double gx, gy;          /* body-force acceleration (Guo forcing), test boxes only */
  int collision;          /* ORACLE_BGK (Eq. 2) or ORACLE_MRT (Eq. 6) */
  double s_rates[9];      /* MRT relaxation rates diag(S); entries 7 and 8 <= 0 mean 1/tau */
  int bounce;             /* cylinder: ORACLE_BB_HALFWAY, ORACLE_BB_INTERP (Sec. 2.4) or
                           * ORACLE_BB_FULLWAY (Sec. 3.1) */
  double q_fixed;         /* interpolated links: > 0 gives every link this wall fraction
                           * (test geometries); else q from the circle of the disk, or 1/2
                           * when the caller supplies the solid mask */
} oracle_params;

typedef struct oracle oracle;

/* Digitise the cylinder: solid iff (2x-cx2)^2 + (2y-cy2)^2 <= D^2, in integers.
 * Writes solid[y*nx+x] in {0,1}.  Returns the number of solid nodes. */
long oracle_digitise(const oracle_params* p, unsigned char* solid);

/* tau from Eqs. 16-17 (nu = U D / Re, tau = 3 nu + 1/2), or p->tau if > 0. */
double oracle_tau(const oracle_params* p);

/* Create a solver.  solid may be NULL (then the digitised disk is used) or a
 * caller array [ny][nx] of 0/1 (copied).  The state is initialised to the
 * equilibrium of rho = 1, u = (U, amp*U*sin(2 pi y/(ny-1))).  NULL on error. */
oracle* oracle_create(const oracle_params* p, const unsigned char* solid);
void oracle_destroy(oracle* o);

/* Advance n steps.  fx, fy (may be NULL) receive the momentum-exchange force
 * on the body computed in each step, from the post-collision populations of
 * that step (Eq. 14).  Returns 0, or 1 + the index of the first step whose
 * density was non-finite or outside (0, 10) (the run stops there). */
long oracle_step(oracle* o, long n, double* fx, double* fy);

long oracle_time(const oracle* o);

/* Macroscopic fields rho, ux, uy [ny][nx] of the current state (Eq. 4).
 * Solid nodes report rho = 1, u = 0. */
void oracle_fields(const oracle* o, double* rho, double* ux, double* uy);

/* State exchange in planar layout [9][ny][nx].
 *  get_f / set_f         : pre-collision state f(t) (after the boundary corrections)
 *  get_fstar / set_fstar : post-collision state f*(t); after set_fstar the next
 *                          step starts at streaming.                          */
void oracle_get_f(const oracle* o, double* out);
void oracle_set_f(oracle* o, const double* in);
void oracle_get_fstar(const oracle* o, double* out);
void oracle_set_fstar(oracle* o, const double* in);

/* The MRT transformation matrix of Sec. 2.1 (row-major 9 x 9) and the
 * moment-space equilibrium m_eq(rho, u, v) the oracle uses, for tests. */
void oracle_mrt_matrix(double* M);
void oracle_mrt_meq(double rho, double ux, double uy, double* meq);

/* Wall fractions q of the links, in the order of the oracle's link list
 * (row-major fluid nodes, directions 1..8): out_node[i] = y*nx + x,
 * out_dir[i] = k (the link from that node along c_k ends in a solid node),
 * out_q[i] = q.  Returns the number of links; arrays may be NULL to count. */
long oracle_links(const oracle* o, long* out_node, int* out_dir, double* out_q);

/* OpenMP threads the oracle's parallel loops use. */
int oracle_threads(void);
void oracle_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
