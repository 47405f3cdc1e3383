/*
 * sanitize_oracle.c -- drives every entry point of the oracle (oracle/ibo.c)
 * on small ragged problems, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_sanitize.py compiles and runs it).
 * Test infrastructure: it checks memory safety and defined behaviour, not
 * values (the pins in tests/test_oracle_*.py do that).  Exit status 0 and a
 * finite checksum on stdout mean every call ran clean.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ibo.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* splitmix64 -> [0, 1) */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static double *field(int64_t n, double amp) {
  double *f = (double *)malloc(sizeof(double) * (size_t)n);
  for (int64_t i = 0; i < n; i++) f[i] = amp * (2.0 * urand() - 1.0);
  return f;
}

static double sum(const double *a, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; i++) s += a[i];
  return s;
}

/* A closed ring of np points joined by zero-rest-length links around the
 * centre of the box, in the (x, y) plane (z = centre in 3-D). */
static void ring(int dim, const double box[3], int64_t np, double *X, int32_t *la, int32_t *lb,
                 double *lk, double *l0) {
  for (int64_t k = 0; k < np; k++) {
    const double t = 2.0 * M_PI * (double)k / (double)np;
    X[0 * np + k] = 0.5 * box[0] + 0.25 * box[0] * cos(t);
    X[1 * np + k] = 0.5 * box[1] + 0.2 * box[1] * sin(t);
    if (dim == 3) X[2 * np + k] = 0.5 * box[2] + 0.1 * box[2] * sin(2 * t);
    la[k] = (int32_t)k;
    lb[k] = (int32_t)((k + 1) % np);
    lk[k] = 0.5 + urand();
    l0[k] = (k % 3 == 0) ? 0.01 : 0.0;
  }
}

static double run_case(int dim, int n0, int n1, int n2, int walls, int noadv, int tethers,
                       int steps) {
  ibo_params P;
  memset(&P, 0, sizeof(P));
  P.dim = dim;
  P.n[0] = n0, P.n[1] = n1, P.n[2] = dim == 3 ? n2 : 1;
  P.h = 1.0 / n0;
  P.rho = 1.3, P.mu = 0.05, P.dt = 1e-3, P.chi = 0.6;
  P.rotate = 1;
  P.no_advection = noadv;
  P.walls_y = walls;
  P.body_force[0] = walls ? 0.5 : 0.1;
  P.wall_velocity[0] = walls ? 0.3 : 0.0; /* a moving upper wall */
  const int64_t nc = (int64_t)P.n[0] * P.n[1] * P.n[2];
  const double box[3] = {n0 * P.h, n1 * P.h, P.n[2] * P.h};
  const int64_t np = 37;
  ibo_sim s;
  memset(&s, 0, sizeof(s));
  s.prm = P;
  for (int c = 0; c < 3; c++) {
    s.u[c] = c < dim ? field(nc, walls ? 0.0 : 0.05) : NULL;
    s.nl_prev[c] = c < dim ? field(nc, 0.0) : NULL;
  }
  s.p = field(nc, 0.0);
  s.psi = field(nc, 0.0);
  s.np = np;
  s.X = (double *)malloc(sizeof(double) * dim * np);
  s.U_prev = field(dim * np, 0.0);
  int32_t *la = (int32_t *)malloc(sizeof(int32_t) * np), *lb = (int32_t *)malloc(sizeof(int32_t) * np);
  double *lk = (double *)malloc(sizeof(double) * np), *l0 = (double *)malloc(sizeof(double) * np);
  ring(dim, box, np, s.X, la, lb, lk, l0);
  double *w = field(np, 0.0);
  for (int64_t k = 0; k < np; k++) w[k] = 1.0 / np;
  double *tk = NULL, *ty = NULL;
  if (tethers) {
    tk = field(np, 0.0);
    ty = (double *)malloc(sizeof(double) * dim * np);
    memcpy(ty, s.X, sizeof(double) * dim * np);
    for (int64_t k = 0; k < np; k += 2) tk[k] = 10.0;
  }
  s.nlinks = np;
  s.link_a = la, s.link_b = lb, s.link_k = lk, s.link_l0 = l0;
  s.w = w;
  s.tether_k = tk, s.tether_Y = ty;
  for (int i = 0; i < steps; i++)
    if (ibo_step(&s) != 0) {
      fprintf(stderr, "ibo_step failed\n");
      exit(2);
    }
  /* the single operators on the same grid */
  double *U = field(dim * np, 0.0), *F = field(dim * np, 0.0);
  double *f[3] = {NULL, NULL, NULL}, *N[3] = {NULL, NULL, NULL}, *g[3] = {NULL, NULL, NULL};
  for (int c = 0; c < dim; c++) f[c] = field(nc, 0.0), N[c] = field(nc, 0.0), g[c] = field(nc, 0.0);
  const double *uc[3] = {s.u[0], s.u[1], s.u[2]};
  ibo_interp(&P, uc, s.X, np, U);
  ibo_link_force(dim, np, s.X, box, np, la, lb, lk, l0, F);
  ibo_link_force(dim, np, s.X, NULL, np, la, lb, lk, l0, F);
  if (tethers) ibo_tether_force(dim, np, s.X, box, tk, ty, F);
  ibo_spread(&P, s.X, F, w, np, f);
  ibo_advection(&P, uc, N);
  double *lap = field(nc, 0.0), *div = field(nc, 0.0);
  ibo_laplacian(&P, s.p, lap);
  for (int c = 0; c < dim; c++) ibo_vel_laplacian(&P, c, s.u[c], lap);
  ibo_divergence(&P, uc, div);
  ibo_gradient(&P, s.p, g);
  int32_t order[3];
  ibo_split_order(&P, 5, order);
  double acc = sum(U, dim * np) + sum(F, dim * np) + sum(lap, nc) + sum(div, nc) + sum(s.p, nc) +
               sum(s.X, dim * np) + order[0];
  for (int c = 0; c < dim; c++) acc += sum(f[c], nc) + sum(N[c], nc) + sum(g[c], nc) + sum(s.u[c], nc);
  for (int c = 0; c < 3; c++) free(s.u[c]), free(s.nl_prev[c]), free(f[c]), free(N[c]), free(g[c]);
  free(s.p), free(s.psi), free(s.X), free(s.U_prev), free(la), free(lb), free(lk), free(l0);
  free(w), free(tk), free(ty), free(U), free(F), free(lap), free(div);
  return acc;
}

static double line_solves(void) {
  double acc = 0.0;
  /* one cyclic system with distinct coefficients */
  for (int n = 3; n <= 9; n++) {
    double *a = field(n, 1.0), *b = field(n, 1.0), *c = field(n, 1.0), *d = field(n, 1.0);
    double *x = field(n, 0.0);
    for (int i = 0; i < n; i++) b[i] = 4.0 + b[i];
    if (ibo_cyclic_solve(n, a, b, c, d, x) != 0) exit(3);
    acc += sum(x, n);
    free(a), free(b), free(c), free(d), free(x);
  }
  /* batched along every axis, every boundary kind, ragged shapes */
  const int32_t shapes[3][3] = {{5, 4, 7}, {9, 6, 3}, {4, 11, 5}};
  for (int sh = 0; sh < 3; sh++) {
    const int64_t nc = (int64_t)shapes[sh][0] * shapes[sh][1] * shapes[sh][2];
    for (int axis = 0; axis < 3; axis++) {
      double *q = field(nc, 1.0);
      if (ibo_line_solve(q, shapes[sh], axis, 3.0, -1.0) != 0) exit(4);
      acc += sum(q, nc);
      for (int bc = 0; bc <= IBO_BC_NEUMANN_CELL; bc++) {
        if (ibo_line_solve_bc(q, shapes[sh], axis, 3.0, -1.0, bc) != 0) exit(5);
        acc += sum(q, nc);
      }
      free(q);
    }
  }
  for (int i = -30; i <= 30; i++) acc += ibo_phi(0.1 * i);
  return acc;
}

int main(void) {
  double acc = line_solves();
  acc += run_case(2, 16, 12, 1, 0, 0, 0, 3);
  acc += run_case(2, 8, 16, 1, 1, 0, 1, 3);   /* channel, tethers */
  acc += run_case(2, 12, 8, 1, 0, 1, 0, 2);   /* Stokes */
  acc += run_case(3, 8, 6, 10, 0, 0, 1, 3);
  acc += run_case(3, 12, 16, 8, 1, 0, 0, 2);  /* 3-D channel */
  if (!isfinite(acc)) {
    fprintf(stderr, "non-finite checksum\n");
    return 6;
  }
  printf("checksum %.17g threads %d\n", acc, ibo_num_threads());
  return 0;
}
