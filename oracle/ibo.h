/*
 * ibo.h -- plain FP64 CPU oracle for the IB-GM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this code: only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the HIP library.
 *
 * It follows the paper (Wiens & Stockie, "An efficient parallel immersed
 * boundary algorithm using a pseudo-compressible fluid solver") step by step:
 *   - Sec. "Discretization of Fluid and IB Domains": MAC grid, Lagrangian grid;
 *   - Sec. "Spatial Finite Difference Operators": D_xx, G^{C->E}, D^{E->C},
 *     D_s^{+-}, and the 4-point delta kernel eq:discretedelta;
 *   - Sec. "IB-GM Algorithm": Steps 1a-1c, 2a-2b, 3a-3f and the n = 0 rules;
 *   - Sec. "Linear Solver": eq:umacstep1/2, eq:PenaltyStepPart1/2, eq:TriDiagX.
 * Every array is FP64.  Grids are stored x fastest: index i + n0*(j + n1*k).
 * Lagrangian arrays are structure-of-arrays: X[a*np + k] is coordinate a of
 * point k.
 */
#ifndef IBO_H
#define IBO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t dim;        /* 2 or 3 */
  int32_t n[3];       /* cells per axis; n[2] = 1 in 2D */
  double h;           /* mesh width; the box is [0, n[a] h) per axis */
  double rho, mu, dt; /* density, viscosity, time step */
  double chi;         /* pressure-correction weight (0.6 in the paper) */
  int32_t rotate;     /* 1: rotate the split order every step */
  int32_t no_advection; /* 1: drop the advection term (Stokes flow) */
  int32_t walls_y;    /* 1: no-slip walls at y = 0 and y = n1 h (a channel,
                         periodic in x and z); 0: periodic in y */
  double body_force[3]; /* uniform force density added to f (0: none) */
  double wall_velocity[3]; /* walls_y: velocity of the upper wall y = n1 h
                              (tangential: x and z; [1] is 0); the lower wall
                              is at rest.  0 without walls */
} ibo_params;

typedef struct {
  ibo_params prm;
  int64_t step;               /* n: number of steps already taken */
  double *u[3];               /* u^n, per component, MAC faces */
  double *nl_prev[3];         /* N(u^{n-1}) (unused at n = 0) */
  double *p;                  /* p^{n-1/2}, cell centres */
  double *psi;                /* psi^{n-1/2}, cell centres */
  int64_t np;                 /* number of Lagrangian points */
  double *X;                  /* X^n   [dim][np], unwrapped coordinates */
  double *U_prev;             /* U^{n-1} [dim][np] (unused at n = 0) */
  int64_t nlinks;             /* elastic links (force connections) */
  const int32_t *link_a, *link_b;
  const double *link_k, *link_l0;
  const double *w;            /* per-point quadrature weight for spreading */
  const double *tether_k;     /* [np] tether stiffness (0: free), or NULL */
  const double *tether_Y;     /* [dim][np] fixed tether targets, or NULL */
} ibo_sim;

/* eq:discretedelta, the 4-point kernel phi(r), written with its two
 * square-root branches. */
double ibo_phi(double r);

/* One cyclic tridiagonal system (eq:TriDiagX with arbitrary coefficients):
 *   a[i] x[i-1] + b[i] x[i] + c[i] x[i+1] = d[i],  indices mod n, n >= 3.
 * Thomas algorithm plus a Sherman-Morrison rank-one correction for the two
 * corner entries.  Returns 0, or -1 on n < 3 / zero pivot. */
int ibo_cyclic_solve(int32_t n, const double *a, const double *b,
                     const double *c, const double *d, double *x);

/* Batched constant-coefficient periodic line solve along one axis, in place:
 * every line of `field` along `axis` is replaced by the solution of
 * (off) x[i-1] + (diag) x[i] + (off) x[i+1] = rhs[i].  Each line goes through
 * ibo_cyclic_solve with no use of the constant coefficients. */
int ibo_line_solve(double *field, const int32_t n[3], int32_t axis,
                   double diag, double off);

/* Step 1a: U_k = sum_ij u_ij delta_h(x_ij - X_k) h^d for each MAC component. */
void ibo_interp(const ibo_params *prm, const double *const u[3],
                const double *X, int64_t np, double *U);

/* Step 2b: f_ij = sum_k F_k delta_h(x_ij - X_k) w_k (f is overwritten). */
void ibo_spread(const ibo_params *prm, const double *X, const double *F,
                const double *w, int64_t np, double *const f[3]);

/* Step 2a in force-connection form: for each link (a, b, kappa, l0),
 * F_a += kappa (X_b - X_a)(1 - l0/|X_b - X_a|) and F_b gets the opposite,
 * X_b - X_a being the nearest periodic image in a box of lengths period[]
 * (NULL: no images). */
void ibo_link_force(int32_t dim, int64_t np, const double *X, const double *period,
                    int64_t nlinks, const int32_t *la, const int32_t *lb,
                    const double *lk, const double *ll0, double *F);

/* Tether points: F_k += kappa_k (Y_k - X_k) towards the fixed target Y_k,
 * nearest periodic image in a box of lengths period[] (NULL: no images). */
void ibo_tether_force(int32_t dim, int64_t np, const double *X, const double *period,
                      const double *kappa, const double *Y, double *F);

/* Skew-symmetric advection N(u) = 1/2 u.grad u + 1/2 div(uu) on the MAC
 * grid with the second-order staggered stencils of Morinishi et al. */
void ibo_advection(const ibo_params *prm, const double *const u[3],
                   double *const N[3]);

/* D_xx + D_yy (+ D_zz) of a field at any fixed staggering (periodic box). */
void ibo_laplacian(const ibo_params *prm, const double *q, double *out);

/* The same for velocity component c, with the channel's no-slip walls when
 * prm->walls_y is set (tangential components reflect oddly across a wall,
 * v is zero on the wall faces). */
void ibo_vel_laplacian(const ibo_params *prm, int32_t c, const double *q, double *out);

/* Line-solve boundary kinds: periodic; Dirichlet for a cell-centred unknown
 * (ghost value -x across the wall); Dirichlet for a face unknown whose
 * element 0 lies on the wall (x_0 = 0, and x_N = 0 on the opposite wall);
 * Neumann for a cell-centred unknown (ghost value +x). */
enum { IBO_BC_PERIODIC = 0, IBO_BC_DIRICHLET_CELL = 1, IBO_BC_DIRICHLET_FACE = 2,
       IBO_BC_NEUMANN_CELL = 3 };

/* eq:TriDiagX along `axis` with the given boundary kind (a plain Thomas
 * solve of the bounded system for the non-periodic kinds). */
int ibo_line_solve_bc(double *field, const int32_t n[3], int32_t axis, double diag,
                      double off, int32_t bc);

/* D^{E->C} . u : forward differences to the cell centres. */
void ibo_divergence(const ibo_params *prm, const double *const u[3],
                    double *out);

/* G^{C->E} p : backward differences to the faces. */
void ibo_gradient(const ibo_params *prm, const double *p, double *const g[3]);

/* Split order used at step n: order[0..dim-1] is a permutation of the axes.
 * Without rotation it is (x, y[, z]); with rotation it is the n-th cyclic
 * shift. */
void ibo_split_order(const ibo_params *prm, int64_t n, int32_t order[3]);

/* One IB-GM time step (Steps 1a-3f), advancing every state array of `s`
 * from n to n+1.  Returns 0, or -1 on invalid parameters / allocation. */
int ibo_step(ibo_sim *s);

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int ibo_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
