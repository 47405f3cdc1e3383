/*
 * ibo.c -- plain FP64 CPU oracle for the IB-GM time step.
 *
 * TEST INFRASTRUCTURE ONLY (see ibo.h).  Written for a reader holding the
 * paper: each function names the section / equation / algorithm step it
 * restates.  No blocking, fusion or reordering beyond what the paper states;
 * OpenMP only splits independent lines / cells / points across threads, so
 * the arithmetic of every output value is the same at any thread count.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes of the repository):
 *   - 3D: the momentum step uses the full 3-D Laplacian explicitly, then one
 *     implicit sweep per axis; the pressure increment uses three sweeps.
 *   - Split-order rotation: at step n the axes are taken in the n-th cyclic
 *     shift of (x, y[, z]); the same order is used for momentum and psi.
 *   - Step 3a: p* = p^{n-1/2} + psi^{n-1/2} at every step; with the initial
 *     state p = psi = 0 this is the paper's n = 0 rule p* = 0.
 *   - The skew-symmetric advection stencil is the second-order staggered one
 *     of Morinishi et al. (1998): 1/2 (divergence form) + 1/2 (advective form).
 *   - The 4-point stencil of a point at xi = X/h - s (s = 0 on the face axis
 *     of a velocity component, 1/2 otherwise) starts at floor(xi) - 1.
 */
#include "ibo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int ibo_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------- grid -- */

static int64_t wrapi(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

static int64_t ncells(const ibo_params *P) {
  return (int64_t)P->n[0] * P->n[1] * P->n[2];
}

/* Value of grid array q at integer cell index (i, j, k), periodic. */
static double at(const ibo_params *P, const double *q, int64_t i, int64_t j,
                 int64_t k) {
  int64_t ii = wrapi(i, P->n[0]), jj = wrapi(j, P->n[1]),
          kk = wrapi(k, P->n[2]);
  return q[ii + (int64_t)P->n[0] * (jj + (int64_t)P->n[1] * kk)];
}

/* Velocity component c at integer index (i, j, k).  Periodic, except across
 * the channel's walls (walls_y): a tangential component (c != 1, stored at
 * cell centres in y) takes the no-slip ghost value of the cell across the
 * wall, -u at the lower wall (at rest) and 2 U_c - u at the upper wall
 * moving with U (so the mean of the two values straddling a wall is the
 * wall's velocity); v (c == 1) is stored on the y faces, face 0 is the wall
 * (both walls, periodically) and holds 0, so plain periodic indexing
 * already gives the wall value there. */
static double vel(const ibo_params *P, int32_t c, const double *q, int64_t i, int64_t j,
                  int64_t k) {
  if (P->walls_y && c != 1) {
    const int64_t n1 = P->n[1];
    if (j < 0) return -at(P, q, i, -1 - j, k);
    if (j >= n1) return 2.0 * P->wall_velocity[c] - at(P, q, i, 2 * n1 - 1 - j, k);
  }
  return at(P, q, i, j, k);
}

static int valid_params(const ibo_params *P) {
  if (P->dim != 2 && P->dim != 3) return 0;
  for (int a = 0; a < P->dim; a++)
    if (P->n[a] < 4) return 0;
  if (P->dim == 2 && P->n[2] != 1) return 0;
  if (!(P->h > 0) || !(P->rho > 0) || !(P->dt > 0) || !(P->mu >= 0))
    return 0;
  /* a wall velocity needs the walls, and is tangential */
  for (int a = 0; a < 3; a++)
    if (P->wall_velocity[a] != 0.0 && (!P->walls_y || a == 1)) return 0;
  return 1;
}

/* ------------------------------------------------------ delta function -- */

/* eq:discretedelta: the two branches exactly as printed. */
double ibo_phi(double r) {
  double a = fabs(r);
  if (a < 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
  if (a < 2.0)
    return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
  return 0.0;
}

/* ------------------------------------------------------- linear solver -- */

/* Non-periodic tridiagonal (Thomas) solve: sub a[1..n-1], diagonal b,
 * super c[0..n-2]. */
static int thomas(int32_t n, const double *a, const double *b, const double *c,
                  const double *d, double *x, double *cp, double *dp) {
  if (b[0] == 0.0) return -1;
  cp[0] = c[0] / b[0];
  dp[0] = d[0] / b[0];
  for (int32_t i = 1; i < n; i++) {
    double m = b[i] - a[i] * cp[i - 1];
    if (m == 0.0) return -1;
    cp[i] = (i < n - 1) ? c[i] / m : 0.0;
    dp[i] = (d[i] - a[i] * dp[i - 1]) / m;
  }
  x[n - 1] = dp[n - 1];
  for (int32_t i = n - 2; i >= 0; i--) x[i] = dp[i] - cp[i] * x[i + 1];
  return 0;
}

/* eq:TriDiagX for one periodic line.  The periodic matrix is written as a
 * non-periodic tridiagonal T plus the rank-one term u v^T carrying the two
 * corner entries a[0] (row 0, column n-1) and c[n-1] (row n-1, column 0):
 *   u = (g, 0, ..., 0, c[n-1]),  v = (1, 0, ..., 0, a[0]/g),  g = -b[0];
 * T has diagonal b with b[0] - g and b[n-1] - c[n-1] a[0]/g in its corners.
 * Sherman-Morrison:  x = y - (v.y / (1 + v.z)) z  with  T y = d,  T z = u. */
int ibo_cyclic_solve(int32_t n, const double *a, const double *b,
                     const double *c, const double *d, double *x) {
  if (n < 3) return -1;
  double g = -b[0];
  if (g == 0.0) return -1;
  double *buf = (double *)malloc(sizeof(double) * 6 * (size_t)n);
  if (!buf) return -1;
  double *bb = buf, *y = buf + n, *z = buf + 2 * n, *uu = buf + 3 * n,
         *cp = buf + 4 * n, *dp = buf + 5 * n;
  for (int32_t i = 0; i < n; i++) {
    bb[i] = b[i];
    uu[i] = 0.0;
  }
  bb[0] = b[0] - g;
  bb[n - 1] = b[n - 1] - c[n - 1] * a[0] / g;
  uu[0] = g;
  uu[n - 1] = c[n - 1];
  int rc = thomas(n, a, bb, c, d, y, cp, dp);
  if (rc == 0) rc = thomas(n, a, bb, c, uu, z, cp, dp);
  if (rc == 0) {
    double vy = y[0] + a[0] / g * y[n - 1];
    double vz = z[0] + a[0] / g * z[n - 1];
    double fac = vy / (1.0 + vz);
    for (int32_t i = 0; i < n; i++) x[i] = y[i] - fac * z[i];
  }
  free(buf);
  return rc;
}

/* eq:TriDiagX batched: every line along `axis` is an independent periodic
 * system with constant coefficients (diag on the diagonal, off on both
 * neighbours).  The coefficients are expanded to full per-row arrays and
 * handed to the generic solver, line by line. */
int ibo_line_solve(double *field, const int32_t n[3], int32_t axis,
                   double diag, double off) {
  if (axis < 0 || axis > 2 || n[0] < 1 || n[1] < 1 || n[2] < 1) return -1;
  const int32_t N = n[axis];
  if (N < 3) return -1;
  const int64_t n0 = n[0], n1 = n[1], n2 = n[2];
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? n0 : n0 * n1);
  const int64_t nlines = n0 * n1 * n2 / N;
  int err = 0;
#pragma omp parallel
  {
    double *buf = (double *)malloc(sizeof(double) * 5 * (size_t)N);
    double *a = buf, *b = buf + N, *c = buf + 2 * N, *d = buf + 3 * N,
           *x = buf + 4 * N;
    if (!buf) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for
    for (int64_t L = 0; L < nlines; L++) {
      if (!buf) continue;
      int64_t base;
      if (axis == 0) base = L * n0;
      else if (axis == 1) base = (L % n0) + (L / n0) * n0 * n1;
      else base = L;
      for (int32_t i = 0; i < N; i++) {
        a[i] = off;
        b[i] = diag;
        c[i] = off;
        d[i] = field[base + i * stride];
      }
      if (ibo_cyclic_solve(N, a, b, c, d, x) != 0) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      for (int32_t i = 0; i < N; i++) field[base + i * stride] = x[i];
    }
    free(buf);
  }
  (void)n2;
  return err ? -1 : 0;
}

/* eq:TriDiagX with the channel's boundary kinds along one axis.  The wall
 * rows are written out: a ghost value -x (Dirichlet, cell-centred) or +x
 * (Neumann, cell-centred) across the wall folds into the diagonal of the
 * first and last rows; a face unknown on the wall (element 0, and element N
 * on the opposite wall) is zero, so rows 1..N-1 form the system.  Each is a
 * plain Thomas solve. */
int ibo_line_solve_bc(double *field, const int32_t n[3], int32_t axis, double diag,
                      double off, int32_t bc) {
  if (bc == IBO_BC_PERIODIC) return ibo_line_solve(field, n, axis, diag, off);
  if (axis < 0 || axis > 2 || bc < 1 || bc > 3) return -1;
  const int32_t N = n[axis];
  if (N < 3) return -1;
  const int64_t n0 = n[0], n1 = n[1], n2 = n[2];
  const int64_t stride = axis == 0 ? 1 : (axis == 1 ? n0 : n0 * n1);
  const int64_t nlines = n0 * n1 * n2 / N;
  int err = 0;
#pragma omp parallel
  {
    double *buf = (double *)malloc(sizeof(double) * 7 * (size_t)N);
    if (!buf) {
#pragma omp atomic write
      err = 1;
    }
#pragma omp for
    for (int64_t L = 0; L < nlines; L++) {
      if (!buf) continue;
      double *a = buf, *b = buf + N, *c = buf + 2 * N, *d = buf + 3 * N, *x = buf + 4 * N,
             *cp = buf + 5 * N, *dp = buf + 6 * N;
      int64_t base;
      if (axis == 0) base = L * n0;
      else if (axis == 1) base = (L % n0) + (L / n0) * n0 * n1;
      else base = L;
      const int32_t first = bc == IBO_BC_DIRICHLET_FACE ? 1 : 0;
      const int32_t m = N - first;
      for (int32_t r = 0; r < m; r++) {
        a[r] = off;
        b[r] = diag;
        c[r] = off;
        d[r] = field[base + (r + first) * stride];
      }
      if (bc == IBO_BC_DIRICHLET_CELL) {
        b[0] = diag - off;
        b[m - 1] = diag - off;
      } else if (bc == IBO_BC_NEUMANN_CELL) {
        b[0] = diag + off;
        b[m - 1] = diag + off;
      }
      if (thomas(m, a, b, c, d, x, cp, dp) != 0) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      if (first) field[base] = 0.0;
      for (int32_t r = 0; r < m; r++) field[base + (r + first) * stride] = x[r];
    }
    free(buf);
  }
  (void)n2;
  return err ? -1 : 0;
}

/* --------------------------------------------------- spread and interp -- */

/* Stencil of one point for MAC component c: base index and 4 weights per
 * axis.  Component c sits at integer positions along axis c and at
 * half-integer positions along the others (Sec. "Discretization of Fluid and
 * IB Domains"); phi((x_a - X_a)/h) = phi(idx - xi). */
static void stencil(const ibo_params *P, int32_t c, const double *Xk_axes,
                    int64_t base[3], double wt[3][4]) {
  for (int32_t a = 0; a < 3; a++) {
    if (a >= P->dim) {
      base[a] = 0;
      wt[a][0] = 1.0;
      wt[a][1] = wt[a][2] = wt[a][3] = 0.0;
      continue;
    }
    double xi = Xk_axes[a] / P->h - (a == c ? 0.0 : 0.5);
    int64_t b = (int64_t)floor(xi) - 1;
    base[a] = b;
    for (int32_t t = 0; t < 4; t++) wt[a][t] = ibo_phi((double)(b + t) - xi);
  }
}

/* Step 1a: U^n_k = sum_ij u^n_ij delta_h(x_ij - X^n_k) h^d.  With
 * delta_h = prod_a phi(.)/h this is the weighted sum over the 4^d stencil. */
void ibo_interp(const ibo_params *P, const double *const u[3], const double *X,
                int64_t np, double *U) {
  const int32_t d = P->dim;
  const int32_t t2max = d == 3 ? 4 : 1;
#pragma omp parallel for
  for (int64_t k = 0; k < np; k++) {
    double Xk[3] = {0, 0, 0};
    for (int32_t a = 0; a < d; a++) Xk[a] = X[a * np + k];
    for (int32_t c = 0; c < d; c++) {
      int64_t base[3];
      double wt[3][4];
      stencil(P, c, Xk, base, wt);
      double s = 0.0;
      for (int32_t t2 = 0; t2 < t2max; t2++)
        for (int32_t t1 = 0; t1 < 4; t1++)
          for (int32_t t0 = 0; t0 < 4; t0++)
            s += at(P, u[c], base[0] + t0, base[1] + t1, base[2] + t2) *
                 wt[0][t0] * wt[1][t1] * wt[2][t2];
      U[c * np + k] = s;
    }
  }
}

/* Step 2b: f_ij = sum_k F_k delta_h(x_ij - X_k) w_k, with delta_h =
 * prod_a phi(.) / h^d.  Serial over points: the sum order is fixed. */
void ibo_spread(const ibo_params *P, const double *X, const double *F,
                const double *w, int64_t np, double *const f[3]) {
  const int32_t d = P->dim;
  const int64_t nc = ncells(P);
  const int32_t t2max = d == 3 ? 4 : 1;
  const double hd = d == 3 ? P->h * P->h * P->h : P->h * P->h;
  for (int32_t c = 0; c < d; c++) memset(f[c], 0, sizeof(double) * (size_t)nc);
  for (int64_t k = 0; k < np; k++) {
    double Xk[3] = {0, 0, 0};
    for (int32_t a = 0; a < d; a++) Xk[a] = X[a * np + k];
    for (int32_t c = 0; c < d; c++) {
      int64_t base[3];
      double wt[3][4];
      stencil(P, c, Xk, base, wt);
      double val = F[c * np + k] * w[k] / hd;
      for (int32_t t2 = 0; t2 < t2max; t2++)
        for (int32_t t1 = 0; t1 < 4; t1++)
          for (int32_t t0 = 0; t0 < 4; t0++) {
            int64_t ii = wrapi(base[0] + t0, P->n[0]);
            int64_t jj = wrapi(base[1] + t1, P->n[1]);
            int64_t kk = wrapi(base[2] + t2, P->n[2]);
            f[c][ii + (int64_t)P->n[0] * (jj + (int64_t)P->n[1] * kk)] +=
                val * wt[0][t0] * wt[1][t1] * wt[2][t2];
          }
    }
  }
}

/* ------------------------------------------------------- elastic force -- */

/* Step 2a in the force-connection form of Sec. "Partitioning of the Eulerian
 * and Lagrangian Grids": each connection pulls its two points together with
 * kappa (X_b - X_a)(1 - l0/|X_b - X_a|).  For a closed fiber with
 * kappa = sigma/h_s^2 and l0 = L h_s this is sigma D_s^-(D_s^+ X (1 - L/|D_s^+
 * X|)) of eq:forceDensityDefinition.  The box is periodic, and a fiber may
 * close through its periodic copy (the axial fibers of Sec. "Cylindrical
 * Shell in 3D"): X_b - X_a is taken as the nearest periodic image, i.e. an
 * integer number of box lengths period[c] is removed from each component
 * (period == NULL: no images). */
void ibo_link_force(int32_t dim, int64_t np, const double *X, const double *period,
                    int64_t nlinks, const int32_t *la, const int32_t *lb,
                    const double *lk, const double *ll0, double *F) {
  memset(F, 0, sizeof(double) * (size_t)(dim * np));
  for (int64_t e = 0; e < nlinks; e++) {
    int64_t a = la[e], b = lb[e];
    double dx[3] = {0, 0, 0}, len2 = 0.0;
    for (int32_t c = 0; c < dim; c++) {
      dx[c] = X[c * np + b] - X[c * np + a];
      if (period) dx[c] -= period[c] * round(dx[c] / period[c]);
      len2 += dx[c] * dx[c];
    }
    double t = lk[e];
    if (ll0[e] != 0.0) t = lk[e] * (1.0 - ll0[e] / sqrt(len2));
    for (int32_t c = 0; c < dim; c++) {
      F[c * np + a] += t * dx[c];
      F[c * np + b] -= t * dx[c];
    }
  }
}

/* Tether points (the paper's route to complex solid boundaries, Sec.
 * "Introduction to the GM method"): a point tied to a fixed target Y by a
 * spring of stiffness kappa feels kappa (Y - X).  Added to F. */
void ibo_tether_force(int32_t dim, int64_t np, const double *X, const double *period,
                      const double *kappa, const double *Y, double *F) {
  for (int64_t k = 0; k < np; k++)
    for (int32_t c = 0; c < dim; c++) {
      double d = Y[c * np + k] - X[c * np + k];
      if (period) d -= period[c] * round(d / period[c]);
      F[c * np + k] += kappa[k] * d;
    }
}

/* ------------------------------------------------ difference operators -- */

/* Skew-symmetric advection, Sec. "IB-GM Algorithm" (Morinishi et al. 1998,
 * second-order staggered).  For component i at its face (i-face of cell c):
 *   Div_i = sum_j delta_j( ubar_j^{x_i} ubar_i^{x_j} ) / h
 *   Adv_i = sum_j avg^{x_j}( ubar_j^{x_i} delta_j u_i / h )
 *   N_i   = 1/2 Div_i + 1/2 Adv_i
 * where ubar^{x} is the two-point average along x and delta_j the one-cell
 * difference along j.  For j = i the products live at cell centres; for
 * j != i they live on the edges shared by u_i and u_j faces. */
void ibo_advection(const ibo_params *P, const double *const u[3],
                   double *const N[3]) {
  const int32_t d = P->dim;
  const double h = P->h;
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
  for (int32_t ci = 0; ci < d; ci++) {
#pragma omp parallel for
    for (int64_t kk = 0; kk < n2; kk++)
      for (int64_t jj = 0; jj < n1; jj++)
        for (int64_t ii = 0; ii < n0; ii++) {
          if (P->walls_y && ci == 1 && jj == 0) {  /* v on the wall: fixed at 0 */
            N[ci][ii + n0 * (jj + n1 * kk)] = 0.0;
            continue;
          }
          int64_t c[3] = {ii, jj, kk};
          int64_t ei[3] = {0, 0, 0};
          ei[ci] = 1;
          double u0 = vel(P, ci, u[ci], c[0], c[1], c[2]);
          double dv = 0.0, ad = 0.0;
          for (int32_t cj = 0; cj < d; cj++) {
            int64_t ej[3] = {0, 0, 0};
            ej[cj] = 1;
            if (cj == ci) {
              double up = vel(P, ci, u[ci], c[0] + ei[0], c[1] + ei[1], c[2] + ei[2]);
              double um = vel(P, ci, u[ci], c[0] - ei[0], c[1] - ei[1], c[2] - ei[2]);
              double ap = 0.5 * (u0 + up); /* centre of cell c */
              double am = 0.5 * (um + u0); /* centre of cell c - e_i */
              dv += (ap * ap - am * am) / h;
              ad += 0.5 * (ap * (up - u0) / h + am * (u0 - um) / h);
            } else {
              /* transporting velocity u_j averaged along x_i, on the edges at
               * c (lower j side) and c + e_j (upper j side) */
              double Uj0 =
                  0.5 * (vel(P, cj, u[cj], c[0] - ei[0], c[1] - ei[1], c[2] - ei[2]) +
                         vel(P, cj, u[cj], c[0], c[1], c[2]));
              double Uj1 =
                  0.5 * (vel(P, cj, u[cj], c[0] + ej[0] - ei[0], c[1] + ej[1] - ei[1],
                            c[2] + ej[2] - ei[2]) +
                         vel(P, cj, u[cj], c[0] + ej[0], c[1] + ej[1], c[2] + ej[2]));
              double ujp = vel(P, ci, u[ci], c[0] + ej[0], c[1] + ej[1], c[2] + ej[2]);
              double ujm = vel(P, ci, u[ci], c[0] - ej[0], c[1] - ej[1], c[2] - ej[2]);
              double ui0 = 0.5 * (ujm + u0); /* u_i averaged along x_j, edge c */
              double ui1 = 0.5 * (u0 + ujp); /* same, edge c + e_j */
              dv += (Uj1 * ui1 - Uj0 * ui0) / h;
              ad += 0.5 * (Uj1 * (ujp - u0) / h + Uj0 * (u0 - ujm) / h);
            }
          }
          N[ci][ii + n0 * (jj + n1 * kk)] = 0.5 * dv + 0.5 * ad;
        }
  }
}

/* Sec. "Spatial Finite Difference Operators": sum of the 3-point second
 * differences D_aa over the active axes. */
void ibo_laplacian(const ibo_params *P, const double *q, double *out) {
  const int32_t d = P->dim;
  const double h2 = P->h * P->h;
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
#pragma omp parallel for
  for (int64_t k = 0; k < n2; k++)
    for (int64_t j = 0; j < n1; j++)
      for (int64_t i = 0; i < n0; i++) {
        double q0 = at(P, q, i, j, k);
        double s = (at(P, q, i + 1, j, k) - 2.0 * q0 + at(P, q, i - 1, j, k)) / h2;
        s += (at(P, q, i, j + 1, k) - 2.0 * q0 + at(P, q, i, j - 1, k)) / h2;
        if (d == 3)
          s += (at(P, q, i, j, k + 1) - 2.0 * q0 + at(P, q, i, j, k - 1)) / h2;
        out[i + n0 * (j + n1 * k)] = s;
      }
}

/* Second difference along one axis only (D_aa) of velocity component c
 * (walls through vel(); v on a wall face gets 0). */
static void second_diff(const ibo_params *P, int32_t c, const double *q, int32_t axis,
                        double *out) {
  const double h2 = P->h * P->h;
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
  int64_t e[3] = {0, 0, 0};
  e[axis] = 1;
#pragma omp parallel for
  for (int64_t k = 0; k < n2; k++)
    for (int64_t j = 0; j < n1; j++)
      for (int64_t i = 0; i < n0; i++)
        out[i + n0 * (j + n1 * k)] =
            (P->walls_y && c == 1 && j == 0)
                ? 0.0
                : (vel(P, c, q, i + e[0], j + e[1], k + e[2]) - 2.0 * vel(P, c, q, i, j, k) +
                   vel(P, c, q, i - e[0], j - e[1], k - e[2])) /
                      h2;
}

void ibo_vel_laplacian(const ibo_params *P, int32_t c, const double *q, double *out) {
  const int64_t nc = ncells(P);
  double *tmp = (double *)malloc(sizeof(double) * (size_t)nc);
  if (!tmp) return;
  for (int64_t i = 0; i < nc; i++) out[i] = 0.0;
  for (int32_t a = 0; a < P->dim; a++) {
    second_diff(P, c, q, a, tmp);
    for (int64_t i = 0; i < nc; i++) out[i] += tmp[i];
  }
  free(tmp);
}

/* D^{E->C} . u = sum_a (u_a[c + e_a] - u_a[c]) / h. */
void ibo_divergence(const ibo_params *P, const double *const u[3],
                    double *out) {
  const int32_t d = P->dim;
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
#pragma omp parallel for
  for (int64_t k = 0; k < n2; k++)
    for (int64_t j = 0; j < n1; j++)
      for (int64_t i = 0; i < n0; i++) {
        double s = (at(P, u[0], i + 1, j, k) - at(P, u[0], i, j, k)) / P->h;
        s += (at(P, u[1], i, j + 1, k) - at(P, u[1], i, j, k)) / P->h;
        if (d == 3) s += (at(P, u[2], i, j, k + 1) - at(P, u[2], i, j, k)) / P->h;
        out[i + n0 * (j + n1 * k)] = s;
      }
}

/* G^{C->E} p = ((p[c] - p[c - e_a]) / h)_a. */
void ibo_gradient(const ibo_params *P, const double *p, double *const g[3]) {
  const int32_t d = P->dim;
  const int64_t n0 = P->n[0], n1 = P->n[1], n2 = P->n[2];
#pragma omp parallel for
  for (int64_t k = 0; k < n2; k++)
    for (int64_t j = 0; j < n1; j++)
      for (int64_t i = 0; i < n0; i++) {
        int64_t c = i + n0 * (j + n1 * k);
        double p0 = at(P, p, i, j, k);
        g[0][c] = (p0 - at(P, p, i - 1, j, k)) / P->h;
        g[1][c] = (p0 - at(P, p, i, j - 1, k)) / P->h;
        if (d == 3) g[2][c] = (p0 - at(P, p, i, j, k - 1)) / P->h;
      }
}

void ibo_split_order(const ibo_params *P, int64_t n, int32_t order[3]) {
  const int32_t d = P->dim;
  int32_t shift = P->rotate ? (int32_t)(n % d) : 0;
  for (int32_t i = 0; i < 3; i++) order[i] = i < d ? (i + shift) % d : i;
}

/* ------------------------------------------------------------ the step -- */

int ibo_step(ibo_sim *s) {
  const ibo_params *P = &s->prm;
  if (!valid_params(P) || s->np < 0 || s->nlinks < 0) return -1;
  const int32_t d = P->dim;
  const int64_t nc = ncells(P), np = s->np;
  const int64_t n = s->step;
  const double dt = P->dt, rho = P->rho, mu = P->mu, h = P->h;

  /* scratch */
  const size_t lag = sizeof(double) * (size_t)(3 * (np > 0 ? np : 1));
  const size_t fld = sizeof(double) * (size_t)nc;
  double *U = (double *)malloc(lag), *Xn1 = (double *)malloc(lag),
         *Xh = (double *)malloc(lag), *F = (double *)malloc(lag);
  double *blk = (double *)malloc(fld * 18);
  if (!U || !Xn1 || !Xh || !F || !blk) {
    free(U); free(Xn1); free(Xh); free(F); free(blk);
    return -1;
  }
  double *f[3], *Nn[3], *un[3], *us[3], *g[3];
  for (int32_t c = 0; c < 3; c++) {
    f[c] = blk + (0 + c) * nc;
    Nn[c] = blk + (3 + c) * nc;
    un[c] = blk + (6 + c) * nc;
    us[c] = blk + (9 + c) * nc;
    g[c] = blk + (12 + c) * nc;
  }
  double *pstar = blk + 15 * nc, *lap = blk + 16 * nc, *rhs = blk + 17 * nc;

  /* Step 1a: interpolate u^n to the points. */
  ibo_interp(P, (const double *const *)s->u, s->X, np, U);

  /* Step 1b: Adams-Bashforth for X (forward Euler at n = 0). */
  for (int64_t i = 0; i < d * np; i++) {
    if (n == 0) Xn1[i] = s->X[i] + dt * U[i];
    else Xn1[i] = s->X[i] + dt * (1.5 * U[i] - 0.5 * s->U_prev[i]);
  }
  /* Step 1c: midpoint position. */
  for (int64_t i = 0; i < d * np; i++) Xh[i] = 0.5 * (Xn1[i] + s->X[i]);

  /* Step 2a: force density at X^{n+1/2}. */
  const double box[3] = {P->n[0] * P->h, P->n[1] * P->h, P->n[2] * P->h};
  ibo_link_force(d, np, Xh, box, s->nlinks, s->link_a, s->link_b, s->link_k,
                 s->link_l0, F);
  if (s->tether_k) ibo_tether_force(d, np, Xh, box, s->tether_k, s->tether_Y, F);
  /* Step 2b: spread it to the grid. */
  ibo_spread(P, Xh, F, s->w, np, f);

  /* Step 3a: pressure predictor p* = p^{n-1/2} + psi^{n-1/2}. */
  for (int64_t i = 0; i < nc; i++) pstar[i] = s->p[i] + s->psi[i];

  /* Step 3b: explicit momentum with AB2 advection (N(u^0) alone at n = 0). */
  for (int32_t c = 0; c < d; c++) memcpy(un[c], s->u[c], fld);
  if (P->no_advection) {
    for (int32_t c = 0; c < d; c++) memset(Nn[c], 0, fld);
  } else {
    ibo_advection(P, (const double *const *)un, Nn);
  }
  ibo_gradient(P, pstar, g);
  for (int32_t c = 0; c < d; c++) {
    ibo_vel_laplacian(P, c, un[c], lap);
    for (int64_t i = 0; i < nc; i++) {
      double Nh = (n == 0) ? Nn[c][i] : 1.5 * Nn[c][i] - 0.5 * s->nl_prev[c][i];
      us[c][i] = un[c][i] + dt * (-Nh + (mu * lap[i] - g[c][i] + f[c][i] + P->body_force[c]) / rho);
    }
  }
  /* channel: v stays zero on the wall faces (row j = 0 of every layer) */
  if (P->walls_y)
    for (int64_t k = 0; k < P->n[2]; k++)
      for (int64_t i = 0; i < P->n[0]; i++) us[1][i + (int64_t)P->n[0] * P->n[1] * k] = 0.0;

  /* Steps 3c-3d (and the z sweep in 3D), eq:umacstep1/2:
   *   (1 - nu D_aa) u^(a) = u^(a-1) - nu D_aa u^n,  nu = mu dt / (2 rho). */
  int32_t order[3];
  ibo_split_order(P, n, order);
  const double nu = mu * dt / (2.0 * rho);
  int rc = 0;
  for (int32_t c = 0; c < d && rc == 0; c++) {
    for (int32_t s_ = 0; s_ < d && rc == 0; s_++) {
      int32_t ax = order[s_];
      second_diff(P, c, un[c], ax, lap);
      for (int64_t i = 0; i < nc; i++) us[c][i] = us[c][i] - nu * lap[i];
      const int32_t bc = (P->walls_y && ax == 1)
                             ? (c == 1 ? IBO_BC_DIRICHLET_FACE : IBO_BC_DIRICHLET_CELL)
                             : IBO_BC_PERIODIC;
      /* a moving upper wall: the unknown's ghost across it is 2 U_c - u, so
       * the row next to it carries the known part 2 nu U_c / h^2 on the
       * right-hand side and the solve keeps its homogeneous condition */
      if (bc == IBO_BC_DIRICHLET_CELL && P->wall_velocity[c] != 0.0) {
        const int64_t n0 = P->n[0], n1 = P->n[1];
        for (int64_t k = 0; k < P->n[2]; k++)
          for (int64_t i = 0; i < n0; i++)
            us[c][i + n0 * ((n1 - 1) + n1 * k)] += 2.0 * nu * P->wall_velocity[c] / (h * h);
      }
      rc = ibo_line_solve_bc(us[c], P->n, ax, 1.0 + 2.0 * nu / (h * h), -nu / (h * h), bc);
    }
  }
  /* us now holds u^{n+1}. */

  /* Step 3e, eq:PenaltyStepPart1/2: (1 - D_aa) ... psi = -(rho/dt) D.u^{n+1},
   * one sweep per axis in the same order. */
  if (rc == 0) {
    ibo_divergence(P, (const double *const *)us, rhs);
    for (int64_t i = 0; i < nc; i++) rhs[i] = -(rho / dt) * rhs[i];
    /* channel: psi takes a homogeneous Neumann condition at the walls */
    for (int32_t s_ = 0; s_ < d && rc == 0; s_++)
      rc = ibo_line_solve_bc(rhs, P->n, order[s_], 1.0 + 2.0 / (h * h), -1.0 / (h * h),
                             (P->walls_y && order[s_] == 1) ? IBO_BC_NEUMANN_CELL
                                                            : IBO_BC_PERIODIC);
  }

  if (rc == 0) {
    /* Step 3f: p^{n+1/2} = p^{n-1/2} + psi - chi mu D.(1/2 (u^{n+1} + u^n)). */
    for (int32_t c = 0; c < d; c++)
      for (int64_t i = 0; i < nc; i++) g[c][i] = 0.5 * (us[c][i] + un[c][i]);
    ibo_divergence(P, (const double *const *)g, lap);
    for (int64_t i = 0; i < nc; i++)
      s->p[i] = s->p[i] + rhs[i] - P->chi * mu * lap[i];
    memcpy(s->psi, rhs, fld);

    /* Advance the state. */
    for (int32_t c = 0; c < d; c++) {
      memcpy(s->u[c], us[c], fld);
      memcpy(s->nl_prev[c], Nn[c], fld);
    }
    memcpy(s->U_prev, U, sizeof(double) * (size_t)(d * np));
    memcpy(s->X, Xn1, sizeof(double) * (size_t)(d * np));
    s->step = n + 1;
  }
  free(U); free(Xn1); free(Xh); free(F); free(blk);
  return rc;
}
