// kernels.h -- gfx950 device code of the IB-GM step (included by ibgm.hip).
//
// Grid arrays are [n2][n1][n0], x fastest.  T is the storage type of the
// grid fields (double, or float under the mixed policy); C is the arithmetic
// type of stencils, spreading and interpolation (== T).  Positions,
// pressure and every line-solve recurrence stay in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibgm {

// ---------------------------------------------------------------- helpers --

__device__ __forceinline__ int64_t floor_mod(int64_t i, int64_t n) {
  int64_t r = i % n;
  return r < 0 ? r + n : r;
}

// Weights of the 4-point kernel of eq:discretedelta for the stencil
// floor(xi)-1 .. floor(xi)+2 given q = xi - floor(xi) in [0, 1).  The four
// branches collapse to one square root s = sqrt(1 + 4q - 4q^2):
//   phi(1+q) = (3-2q-s)/8, phi(q) = (3-2q+s)/8,
//   phi(1-q) = (1+2q+s)/8, phi(2-q) = (1+2q-s)/8.
template <typename C>
__device__ __forceinline__ void delta_weights(C q, C w[4]) {
  C s = sqrt(C(1) + C(4) * q - C(4) * q * q);
  w[0] = (C(3) - C(2) * q - s) * C(0.125);
  w[1] = (C(3) - C(2) * q + s) * C(0.125);
  w[2] = (C(1) + C(2) * q + s) * C(0.125);
  w[3] = (C(1) + C(2) * q - s) * C(0.125);
}

// Stencil start (wrapped) and weights along one axis for a point coordinate
// x (physical, unwrapped) and staggering offset s (0 on the face axis of a
// velocity component, 1/2 otherwise).
template <typename C>
__device__ __forceinline__ int64_t axis_stencil(double x, double inv_h, double s,
                                                int64_t n, C w[4]) {
  double xi = x * inv_h - s;
  // A non-finite or absurdly large coordinate must not become an index: it
  // is pinned to cell 0 and its NaN weights carry the failure forward.
  if (!(fabs(xi) < 1e15)) xi = __builtin_nan("");
  double fl = isnan(xi) ? 0.0 : floor(xi);
  delta_weights<C>((C)(xi - fl), w);
  return floor_mod((int64_t)fl - 1, n);
}

struct Grid {
  int32_t n0, n1, n2;
  int64_t ncell;
};

// ------------------------------------------------- Lagrangian: Step 1a-1c --

// One thread per (point, component): interpolate component c of u at X^n
// (Step 1a) and, if `evolve`, advance that coordinate with AB2 (forward
// Euler when `first`) to X^{n+1} and the midpoint X^{n+1/2} (Steps 1b-1c).
template <typename T, int DIM>
struct InterpArgs {
  const T *u[3];
  const double *X;    // [DIM][np]
  double *U;          // [DIM][np]  interpolated velocity (or U^{n-1} in place)
  double *Xn1, *Xh;   // [DIM][np]  (evolve only)
  int *flag;          // set to 1 on a non-finite X^{n+1}
  int64_t np;
  Grid g;
  double inv_h, dt;
  int evolve, first;
};

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_interp(InterpArgs<T, DIM> a) {
  using C = T;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= a.np) return;
  const int32_t nn[3] = {a.g.n0, a.g.n1, a.g.n2};
  C w[3][4];
  int64_t b[3];
  for (int ax = 0; ax < DIM; ax++)
    b[ax] = axis_stencil<C>(a.X[ax * a.np + k], a.inv_h, ax == c ? 0.0 : 0.5,
                            nn[ax], w[ax]);
  const T *__restrict__ uc = a.u[c];
  C acc = 0;
  if (DIM == 3) {
    for (int t2 = 0; t2 < 4; t2++) {
      int64_t kk = b[2] + t2;
      kk -= kk >= nn[2] ? nn[2] : 0;
      C acc1 = 0;
      for (int t1 = 0; t1 < 4; t1++) {
        int64_t jj = b[1] + t1;
        jj -= jj >= nn[1] ? nn[1] : 0;
        const T *row = uc + (kk * nn[1] + jj) * nn[0];
        C acc0 = 0;
        for (int t0 = 0; t0 < 4; t0++) {
          int64_t ii = b[0] + t0;
          ii -= ii >= nn[0] ? nn[0] : 0;
          acc0 += (C)row[ii] * w[0][t0];
        }
        acc1 += acc0 * w[1][t1];
      }
      acc += acc1 * w[2][t2];
    }
  } else {
    for (int t1 = 0; t1 < 4; t1++) {
      int64_t jj = b[1] + t1;
      jj -= jj >= nn[1] ? nn[1] : 0;
      const T *row = uc + jj * nn[0];
      C acc0 = 0;
      for (int t0 = 0; t0 < 4; t0++) {
        int64_t ii = b[0] + t0;
        ii -= ii >= nn[0] ? nn[0] : 0;
        acc0 += (C)row[ii] * w[0][t0];
      }
      acc += acc0 * w[1][t1];
    }
  }
  const double U = (double)acc;
  const int64_t o = c * a.np + k;
  if (!a.evolve) {
    a.U[o] = U;
    return;
  }
  const double x = a.X[o];
  const double xn1 = a.first ? x + a.dt * U : x + a.dt * (1.5 * U - 0.5 * a.U[o]);
  a.U[o] = U;
  a.Xn1[o] = xn1;
  a.Xh[o] = 0.5 * (xn1 + x);
  if (!isfinite(xn1)) *a.flag = 1;
}

// ----------------------------------------------------- Lagrangian: Step 2a --

// One thread per point: gather the link forces at X^{n+1/2} over the point's
// incident links (CSR by point), F_k = sum kappa (X_l - X_k)(1 - l0/|X_l - X_k|).
// When Xn1 != null also commit X <- X^{n+1} for the point.
template <int DIM>
struct ForceArgs {
  const int32_t *ptr, *nbr;
  const double *kap, *l0;
  const double *Xh;
  double *F;
  const double *Xn1;
  double *X;
  int64_t np;
};

template <int DIM>
__global__ void __launch_bounds__(256) k_force(ForceArgs<DIM> a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.np) return;
  double xk[DIM], f[DIM];
  for (int c = 0; c < DIM; c++) {
    xk[c] = a.Xh[c * a.np + k];
    f[c] = 0.0;
  }
  const int32_t e0 = a.ptr[k], e1 = a.ptr[k + 1];
  for (int32_t e = e0; e < e1; e++) {
    const int64_t l = a.nbr[e];
    double d[DIM], len2 = 0.0;
    for (int c = 0; c < DIM; c++) {
      d[c] = a.Xh[c * a.np + l] - xk[c];
      len2 += d[c] * d[c];
    }
    double t = a.kap[e];
    const double r0 = a.l0[e];
    if (r0 != 0.0) t *= 1.0 - r0 / sqrt(len2);
    for (int c = 0; c < DIM; c++) f[c] += t * d[c];
  }
  for (int c = 0; c < DIM; c++) a.F[c * a.np + k] = f[c];
  if (a.Xn1)
    for (int c = 0; c < DIM; c++) a.X[c * a.np + k] = a.Xn1[c * a.np + k];
}

// ----------------------------------------------------- Lagrangian: Step 2b --

// One thread per (point, stencil row): the row is a (y[, z]) offset of the
// 4^DIM support; the thread adds the 4 x-neighbours of every component with
// device atomics.  val = F_c w_k / h^d times the tensor-product weights.
template <typename T, int DIM>
struct SpreadArgs {
  const double *X, *F, *w;
  T *f[3];
  int64_t np;
  Grid g;
  double inv_h, inv_hd;
};

template <typename T>
__device__ __forceinline__ void atomic_add_grid(T *p, T v) {
  unsafeAtomicAdd(p, v);
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_spread(SpreadArgs<T, DIM> a) {
  using C = T;
  constexpr int ROWS = DIM == 3 ? 16 : 4;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = tid / ROWS;
  const int row = (int)(tid % ROWS);
  if (k >= a.np) return;
  const int t1 = row & 3, t2 = row >> 2;
  const int32_t nn[3] = {a.g.n0, a.g.n1, a.g.n2};
  double xk[DIM];
  for (int ax = 0; ax < DIM; ax++) xk[ax] = a.X[ax * a.np + k];
  const double wk = a.w[k] * a.inv_hd;
  for (int c = 0; c < DIM; c++) {
    C w0[4], w1[4], w2[4];
    int64_t b0 = axis_stencil<C>(xk[0], a.inv_h, c == 0 ? 0.0 : 0.5, nn[0], w0);
    int64_t b1 = axis_stencil<C>(xk[1], a.inv_h, c == 1 ? 0.0 : 0.5, nn[1], w1);
    int64_t jj = b1 + t1;
    jj -= jj >= nn[1] ? nn[1] : 0;
    C rw = w1[t1];
    int64_t kk = 0;
    if (DIM == 3) {
      int64_t b2 = axis_stencil<C>(xk[2], a.inv_h, c == 2 ? 0.0 : 0.5, nn[2], w2);
      kk = b2 + t2;
      kk -= kk >= nn[2] ? nn[2] : 0;
      rw *= w2[t2];
    }
    const C val = (C)(a.F[c * a.np + k] * wk) * rw;
    T *row_ptr = a.f[c] + (kk * nn[1] + jj) * nn[0];
    for (int t0 = 0; t0 < 4; t0++) {
      int64_t ii = b0 + t0;
      ii -= ii >= nn[0] ? nn[0] : 0;
      atomic_add_grid<T>(row_ptr + ii, (T)(val * w0[t0]));
    }
  }
}

// ------------------------------------------ Eulerian: Steps 3a-3b fused --

// One thread per cell.  For each component c at its face:
//   N_c  = skew advection (Morinishi 2nd-order staggered: 1/2 divergence form
//          + 1/2 advective form),
//   Nh   = 3/2 N_c - 1/2 N_c^{n-1}   (N_c alone at n = 0),
//   d*_c = dt ( -Nh + (mu Lap u_c - G_c p* + f_c)/rho ),  p* = p + psi (FP64),
// and stores d*_c (the delta-form right-hand side of the first sweep),
// N_c into nl (for the next step) and clears f_c for the next spreading.
template <typename T, int DIM>
struct ExplicitArgs {
  const T *u[3];
  T *nl[3];
  T *f[3];
  T *delta[3];
  const double *p;
  const T *psi;
  Grid g;
  double inv_h, inv_h2, dt, mu, inv_rho;
  int first, advect;
};

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_explicit(ExplicitArgs<T, DIM> a) {
  using C = T;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.g.ncell) return;
  const int64_t n0 = a.g.n0, n1 = a.g.n1, n2 = a.g.n2;
  const int64_t i = idx % n0, j = (idx / n0) % n1, k = idx / (n0 * n1);
  // linear offsets to the +/- neighbour along each axis, periodic
  int64_t dp[3], dm[3];
  dp[0] = (i + 1 == n0) ? -(n0 - 1) : 1;
  dm[0] = (i == 0) ? (n0 - 1) : -1;
  dp[1] = (j + 1 == n1) ? -(n1 - 1) * n0 : n0;
  dm[1] = (j == 0) ? (n1 - 1) * n0 : -n0;
  if (DIM == 3) {
    dp[2] = (k + 1 == n2) ? -(n2 - 1) * n0 * n1 : n0 * n1;
    dm[2] = (k == 0) ? (n2 - 1) * n0 * n1 : -n0 * n1;
  } else {
    dp[2] = dm[2] = 0;
  }
  const double ps0 = a.p[idx] + (double)a.psi[idx];
#pragma unroll
  for (int ci = 0; ci < DIM; ci++) {
    const T *__restrict__ ui = a.u[ci];
    const C u0 = (C)ui[idx];
    C dv = 0, ad = 0, lap = 0;
#pragma unroll
    for (int cj = 0; cj < DIM; cj++) {
      const C up = (C)ui[idx + dp[cj]], um = (C)ui[idx + dm[cj]];
      lap += up - C(2) * u0 + um;
      if (!a.advect) continue;
      if (cj == ci) {
        const C ap = C(0.5) * (u0 + up), am = C(0.5) * (um + u0);
        dv += ap * ap - am * am;
        ad += C(0.5) * (ap * (up - u0) + am * (u0 - um));
      } else {
        const T *__restrict__ uj = a.u[cj];
        const C Uj0 = C(0.5) * ((C)uj[idx + dm[ci]] + (C)uj[idx]);
        const C Uj1 = C(0.5) * ((C)uj[idx + dp[cj] + dm[ci]] + (C)uj[idx + dp[cj]]);
        dv += Uj1 * C(0.5) * (u0 + up) - Uj0 * C(0.5) * (um + u0);
        ad += C(0.5) * (Uj1 * (up - u0) + Uj0 * (u0 - um));
      }
    }
    const C N = C(0.5) * (dv + ad) * (C)a.inv_h;
    const double psm = a.p[idx + dm[ci]] + (double)a.psi[idx + dm[ci]];
    const C gp = (C)((ps0 - psm) * a.inv_h);
    const C Nh = a.first ? N : C(1.5) * N - C(0.5) * (C)a.nl[ci][idx];
    const C fc = (C)a.f[ci][idx];
    const C d = (C)a.dt * (-Nh + ((C)a.mu * lap * (C)a.inv_h2 - gp + fc) * (C)a.inv_rho);
    a.delta[ci][idx] = (T)d;
    a.nl[ci][idx] = (T)N;
    a.f[ci][idx] = (T)0;
  }
}

// D.u at every cell (used once, to seed div_prev = D.u^0).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_divergence(const T *u0, const T *u1,
                                                     const T *u2, T *out, Grid g,
                                                     double inv_h) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.ncell) return;
  const int64_t n0 = g.n0, n1 = g.n1, n2 = g.n2;
  const int64_t i = idx % n0, j = (idx / n0) % n1, k = idx / (n0 * n1);
  double s = (double)u0[idx + ((i + 1 == n0) ? -(n0 - 1) : 1)] - (double)u0[idx];
  s += (double)u1[idx + ((j + 1 == n1) ? -(n1 - 1) * n0 : n0)] - (double)u1[idx];
  if (DIM == 3)
    s += (double)u2[idx + ((k + 1 == n2) ? -(n2 - 1) * n0 * n1 : n0 * n1)] -
         (double)u2[idx];
  out[idx] = (T)(s * inv_h);
}

// ------------------------------------------------------------ line solves --
//
// Every system is the periodic constant-coefficient tridiagonal
//   A = d I + e (L + U),   (L x)_i = x_{i-1},  (U x)_i = x_{i+1}  (mod N),
// with |d| > 2|e|.  It factors exactly as A = c (I - alpha L)(I - alpha U)
// with alpha + 1/alpha = -d/e, |alpha| < 1, c = -e/alpha (host, FP64), so
// A x = b is two periodic first-order recurrences:
//   forward   w_i = alpha w_{i-1} + b_i / c,
//   backward  x_i = alpha x_{i+1} + w_i.
// Each thread owns a contiguous chunk of a line.  It runs the recurrence from
// zero over its chunk, which makes the chunk an affine map v -> A v + B of
// the value entering it; the maps of all chunks are composed (a scan), the
// periodic fixed point v = B_tot / (1 - A_tot) closes the line, and each
// chunk adds alpha^k times its true incoming value.  This is the paper's
// Schur-complement partition of a periodic line (Sec. "Linear Solver") with
// the P x P interface system replaced by the scan of the factored form.

enum { SW_PLAIN = 0, SW_FINAL = 1, SW_DIV = 2, SW_PFINAL = 3 };

template <typename T>
struct SweepArgs {
  T *f[3];             // per field: rhs in, solution out (PLAIN); rhs (FINAL);
                       // psi out (DIV); psi in/out (PFINAL)
  T *u[3];             // FINAL: u += x (per field);  DIV: velocity components
  T *divn;             // DIV: D.u^{n+1} out;  PFINAL: in
  T *divp;             // PFINAL: D.u^n in, D.u^{n+1} out
  double *p;           // PFINAL: p += x - chi mu (divn + divp)/2
  double alpha, inv_c; // factored-form coefficients
  double inv_h;        // DIV: D.u = inv_h * (sum of one-cell differences)
  double div_scale;    // DIV: rhs = -(rho/dt) D.u = div_scale * (sum of differences)
  double half_chi_mu;  // PFINAL
  Grid g;
  int32_t G;           // threads per line (x kernel: power of two <= 64)
  int32_t dim;
};

template <typename T, int MODE>
__device__ __forceinline__ double sweep_load(const SweepArgs<T> &a, int fld,
                                             int64_t idx, int64_t i, int64_t j,
                                             int64_t k) {
  if (MODE == SW_DIV) {
    const int64_t n0 = a.g.n0, n1 = a.g.n1, n2 = a.g.n2;
    double s = (double)a.u[0][idx + ((i + 1 == n0) ? -(n0 - 1) : 1)] - (double)a.u[0][idx];
    s += (double)a.u[1][idx + ((j + 1 == n1) ? -(n1 - 1) * n0 : n0)] - (double)a.u[1][idx];
    if (a.dim == 3)
      s += (double)a.u[2][idx + ((k + 1 == n2) ? -(n2 - 1) * n0 * n1 : n0 * n1)] -
           (double)a.u[2][idx];
    return s;
  } else {
    return (double)a.f[fld][idx];
  }
}

template <typename T, int MODE>
__device__ __forceinline__ void sweep_store(const SweepArgs<T> &a, int fld,
                                            int64_t idx, double x) {
  if (MODE == SW_PLAIN || MODE == SW_DIV) {
    a.f[fld][idx] = (T)x;
  } else if (MODE == SW_FINAL) {
    a.u[fld][idx] = (T)((double)a.u[fld][idx] + x);
  } else {  // SW_PFINAL
    a.f[fld][idx] = (T)x;
    const T dn = a.divn[idx];
    const double dsum = (double)dn + (double)a.divp[idx];
    a.p[idx] = a.p[idx] + x - a.half_chi_mu * dsum;
    a.divp[idx] = dn;
  }
}

// Contiguous (x) lines.  blockDim = 256; G lanes per line (power of two
// <= 64), each with a chunk of M consecutive elements; 256/G lines per block;
// blockIdx.y = field.  Chunks beyond the line end are empty (identity maps).
template <typename T, int M, int MODE>
__global__ void __launch_bounds__(256) k_sweep_x(SweepArgs<T> a) {
  const int G = a.G;
  const int lane = threadIdx.x & (G - 1);
  const int64_t N = a.g.n0;
  const int64_t nlines = (int64_t)a.g.n1 * a.g.n2;
  int64_t line = (int64_t)blockIdx.x * (256 / G) + threadIdx.x / G;
  const bool live = line < nlines;
  if (!live) line = nlines - 1;  // keep the lanes in the shuffles, store nothing
  const int fld = blockIdx.y;
  const int64_t s = (int64_t)lane * M;
  const int cnt = (int)(s >= N ? 0 : (N - s < M ? N - s : M));
  const int64_t base = line * N;
  const int64_t jl = line % a.g.n1, kl = line / a.g.n1;
  const double al = a.alpha, ic = a.inv_c;

  double r[M];
#pragma unroll
  for (int q = 0; q < M; q++) {
    r[q] = 0.0;
    if (q < cnt) {
      double v = sweep_load<T, MODE>(a, fld, base + s + q, s + q, jl, kl);
      if (MODE == SW_DIV) {
        if (live) a.divn[base + s + q] = (T)(v * a.inv_h);
        v *= a.div_scale;
      }
      r[q] = v;
    }
  }
  // forward recurrence over the chunk from zero
  double z = 0.0, A = 1.0;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (q < cnt) {
      z = al * z + r[q] * ic;
      r[q] = z;
      A *= al;
    }
  double B = z;
  // inclusive scan of the affine maps (earlier lanes act first)
  for (int off = 1; off < G; off <<= 1) {
    const double Ap = __shfl_up(A, off, G), Bp = __shfl_up(B, off, G);
    if (lane >= off) {
      B = A * Bp + B;
      A = A * Ap;
    }
  }
  {
    const double At = __shfl(A, G - 1, G), Bt = __shfl(B, G - 1, G);
    const double wlast = Bt / (1.0 - At);
    double Ae = __shfl_up(A, 1, G), Be = __shfl_up(B, 1, G);
    if (lane == 0) {
      Ae = 1.0;
      Be = 0.0;
    }
    const double win = Ae * wlast + Be;
    double pw = al;
#pragma unroll
    for (int q = 0; q < M; q++)
      if (q < cnt) {
        r[q] += pw * win;
        pw *= al;
      }
  }
  // backward recurrence over the chunk from zero
  double t = 0.0;
  A = 1.0;
#pragma unroll
  for (int q = M - 1; q >= 0; q--)
    if (q < cnt) {
      t = al * t + r[q];
      r[q] = t;
      A *= al;
    }
  B = t;
  // suffix scan (later lanes act first)
  for (int off = 1; off < G; off <<= 1) {
    const double An = __shfl_down(A, off, G), Bn = __shfl_down(B, off, G);
    if (lane + off < G) {
      B = A * Bn + B;
      A = A * An;
    }
  }
  {
    const double A0 = __shfl(A, 0, G), B0 = __shfl(B, 0, G);
    const double x0 = B0 / (1.0 - A0);
    double An = __shfl_down(A, 1, G), Bn = __shfl_down(B, 1, G);
    if (lane == G - 1) {
      An = 1.0;
      Bn = 0.0;
    }
    const double xin = An * x0 + Bn;
    double pw = al;
#pragma unroll
    for (int q = M - 1; q >= 0; q--)
      if (q < cnt) {
        r[q] += pw * xin;
        pw *= al;
      }
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (q < cnt) sweep_store<T, MODE>(a, fld, base + s + q, r[q]);
}

// Strided (y or z) lines.  blockDim = (TX, G): threadIdx.x walks TX
// consecutive x (coalesced rows), threadIdx.y = chunk of M consecutive line
// elements (G = ceil(N/M) chunks).  blockIdx.x = x tile, blockIdx.y = the
// remaining axis index, blockIdx.z = field.  Chunk maps are combined through
// LDS.  LB bounds TX*G so that the M-element chunk stays in registers.
template <typename T, int M, int MODE, int LB>
__global__ void __launch_bounds__(LB) k_sweep_s(SweepArgs<T> a, int axis) {
  __shared__ double sA[LB], sB[LB];
  const int TX = blockDim.x, G = blockDim.y;
  const int tx = threadIdx.x, g = threadIdx.y;
  const int64_t n0 = a.g.n0, n1 = a.g.n1;
  const int64_t x = (int64_t)blockIdx.x * TX + tx;
  const bool live = x < n0;
  const int64_t xs = live ? x : n0 - 1;
  const int64_t other = blockIdx.y;
  const int fld = blockIdx.z;
  const int64_t N = axis == 1 ? n1 : a.g.n2;
  const int64_t stride = axis == 1 ? n0 : n0 * n1;
  const int64_t s = (int64_t)g * M;
  const int64_t base = (axis == 1 ? xs + other * n0 * n1 : xs + other * n0) + s * stride;
  const int cnt = (int)(s >= N ? 0 : (N - s < M ? N - s : M));
  const double al = a.alpha, ic = a.inv_c;
  const int slot = g * TX + tx;

  double r[M];
#pragma unroll
  for (int q = 0; q < M; q++) {
    r[q] = 0.0;
    if (q < cnt) {
      const int64_t idx = base + q * stride;
      double v;
      if (MODE == SW_DIV) {
        const int64_t pos = s + q;
        v = sweep_load<T, MODE>(a, fld, idx, xs, axis == 1 ? pos : other,
                                axis == 1 ? other : pos);
        if (live) a.divn[idx] = (T)(v * a.inv_h);
        v *= a.div_scale;
      } else {
        v = (double)a.f[fld][idx];
      }
      r[q] = v;
    }
  }
  double z = 0.0, A = 1.0;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (q < cnt) {
      z = al * z + r[q] * ic;
      r[q] = z;
      A *= al;
    }
  sA[slot] = A;
  sB[slot] = z;
  __syncthreads();
  {
    double Ap = 1.0, Bp = 0.0;  // composite of chunks 0..g-1
    for (int h = 0; h < g; h++) {
      Bp = sA[h * TX + tx] * Bp + sB[h * TX + tx];
      Ap = sA[h * TX + tx] * Ap;
    }
    double At = Ap, Bt = Bp;  // continue to the full line
    for (int h = g; h < G; h++) {
      Bt = sA[h * TX + tx] * Bt + sB[h * TX + tx];
      At = sA[h * TX + tx] * At;
    }
    const double win = Ap * (Bt / (1.0 - At)) + Bp;
    double pw = al;
#pragma unroll
    for (int q = 0; q < M; q++)
      if (q < cnt) {
        r[q] += pw * win;
        pw *= al;
      }
  }
  __syncthreads();
  double t = 0.0;
  A = 1.0;
#pragma unroll
  for (int q = M - 1; q >= 0; q--)
    if (q < cnt) {
      t = al * t + r[q];
      r[q] = t;
      A *= al;
    }
  sA[slot] = A;
  sB[slot] = t;
  __syncthreads();
  {
    double As = 1.0, Bs = 0.0;  // composite of chunks g+1..G-1
    for (int h = G - 1; h > g; h--) {
      Bs = sA[h * TX + tx] * Bs + sB[h * TX + tx];
      As = sA[h * TX + tx] * As;
    }
    double At = As, Bt = Bs;
    for (int h = g; h >= 0; h--) {
      Bt = sA[h * TX + tx] * Bt + sB[h * TX + tx];
      At = sA[h * TX + tx] * At;
    }
    const double xin = As * (Bt / (1.0 - At)) + Bs;
    double pw = al;
#pragma unroll
    for (int q = M - 1; q >= 0; q--)
      if (q < cnt) {
        r[q] += pw * xin;
        pw *= al;
      }
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (q < cnt) sweep_store<T, MODE>(a, fld, base + q * stride, r[q]);
}

}  // namespace ibgm
