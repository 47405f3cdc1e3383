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

// Periodic wrap of a cell index b (any sign, |b| < 2^24) into [0, n).
__device__ __forceinline__ int wrap_cell(int b, int n) {
  b -= n * (int)floorf((float)b / (float)n);
  b += b < 0 ? n : 0;
  b -= b >= n ? n : 0;
  return b;
}

// Stencil start (wrapped) and weights along one axis for a point coordinate
// x (physical, unwrapped) and staggering offset s (0 on the face axis of a
// velocity component, 1/2 otherwise).
template <typename C>
__device__ __forceinline__ int axis_stencil(double x, double inv_h, double s, int n, C w[4]) {
  double xi = x * inv_h - s;
  // A non-finite or absurdly large coordinate must not become an index: it
  // is pinned to cell 0 and its NaN weights carry the failure forward.
  if (!(fabs(xi) < 1e7)) xi = __builtin_nan("");
  double fl = isnan(xi) ? 0.0 : floor(xi);
  delta_weights<C>((C)(xi - fl), w);
  return wrap_cell((int)fl - 1, n);
}

// ----------------------------------------------------- wave-level scans --
//
// Affine maps v -> A v + B, the chunk summaries of the line-solve scans.
// after(f, g) is "f, then g".

struct Aff {
  double A, B;
};

__device__ __forceinline__ Aff after(Aff f, Aff g) { return {g.A * f.A, g.A * f.B + g.B}; }

// Move a double across lanes with a DPP row shift (CTRL = 0x110|n: row_shr n,
// 0x100|n: row_shl n); lanes whose source falls outside their 16-lane row
// receive `ident`.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v, double ident) {
  const int lo = __builtin_amdgcn_update_dpp(__double2loint(ident), __double2loint(v), CTRL,
                                             0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(__double2hiint(ident), __double2hiint(v), CTRL,
                                             0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ Aff dpp_aff(Aff f) {
  return {dpp_move<CTRL>(f.A, 1.0), dpp_move<CTRL>(f.B, 0.0)};
}

__device__ __forceinline__ Aff readlane_aff(Aff f, int lane) {
  const int alo = __builtin_amdgcn_readlane(__double2loint(f.A), lane);
  const int ahi = __builtin_amdgcn_readlane(__double2hiint(f.A), lane);
  const int blo = __builtin_amdgcn_readlane(__double2loint(f.B), lane);
  const int bhi = __builtin_amdgcn_readlane(__double2hiint(f.B), lane);
  return {__hiloint2double(ahi, alo), __hiloint2double(bhi, blo)};
}

// Over segments of SEG = 64 or 32 lanes (a wave holds 64/SEG independent
// lines), lane l holding chunk l's map: the composite of the chunks before l
// in its segment (the segment's first chunk acting first) and of the whole
// segment.  Row-local Hillis-Steele steps use DPP row shifts; the 16-lane
// row totals are read back with readlane and chained.  Requires all 64
// lanes active.
template <int SEG>
__device__ __forceinline__ void wave_prefix(Aff f, Aff &excl, Aff &tot) {
  Aff x = f;
  x = after(dpp_aff<0x111>(x), x);
  x = after(dpp_aff<0x112>(x), x);
  x = after(dpp_aff<0x114>(x), x);
  x = after(dpp_aff<0x118>(x), x);
  const Aff r0 = readlane_aff(x, 15), r1 = readlane_aff(x, 31), r2 = readlane_aff(x, 47),
            r3 = readlane_aff(x, 63);
  const Aff e = dpp_aff<0x111>(x);  // exclusive within the row
  const int row = __lane_id() >> 4;
  Aff pr;
  if (SEG == 64) {
    const Aff p2 = after(r0, r1), p3 = after(p2, r2);
    tot = after(p3, r3);
    pr = row == 0 ? Aff{1.0, 0.0} : (row == 1 ? r0 : (row == 2 ? p2 : p3));
  } else {
    const bool hi = row >= 2;
    tot = hi ? after(r2, r3) : after(r0, r1);
    pr = (row & 1) == 0 ? Aff{1.0, 0.0} : (hi ? r2 : r0);
  }
  excl = after(pr, e);
}

// Mirror image for maps acting right to left (the segment's last chunk
// first): the composite of the chunks after l in its segment, and of all.
template <int SEG>
__device__ __forceinline__ void wave_suffix(Aff f, Aff &excl, Aff &tot) {
  Aff x = f;
  x = after(dpp_aff<0x101>(x), x);
  x = after(dpp_aff<0x102>(x), x);
  x = after(dpp_aff<0x104>(x), x);
  x = after(dpp_aff<0x108>(x), x);
  const Aff t0 = readlane_aff(x, 0), t1 = readlane_aff(x, 16), t2 = readlane_aff(x, 32),
            t3 = readlane_aff(x, 48);
  const Aff e = dpp_aff<0x101>(x);  // exclusive within the row
  const int row = __lane_id() >> 4;
  Aff qr;
  if (SEG == 64) {
    const Aff q1 = after(t3, t2), q0 = after(q1, t1);
    tot = after(q0, t0);
    qr = row == 3 ? Aff{1.0, 0.0} : (row == 2 ? t3 : (row == 1 ? q1 : q0));
  } else {
    const bool hi = row >= 2;
    tot = hi ? after(t3, t2) : after(t1, t0);
    qr = (row & 1) == 1 ? Aff{1.0, 0.0} : (hi ? t3 : t1);
  }
  excl = after(qr, e);
}

struct Grid {
  int32_t n0, n1, n2;
  int64_t ncell;
};

// ------------------------------------------------- Lagrangian: Step 1a-1c --

// Four lanes per (point, component): interpolate component c of u at X^n
// (Step 1a) and, if `evolve`, advance that coordinate with AB2 (forward
// Euler when `first`) to X^{n+1} and the midpoint X^{n+1/2} (Steps 1b-1c).
template <typename T, int DIM>
struct InterpArgs {
  const T *u[3];
  const double *X;    // [DIM][np]
  double *U;          // [DIM][np]  interpolated velocity (or U^{n-1} in place)
  double *Xn1, *Xh;   // [DIM][np]  (evolve only)
  int *flag;          // set to 1 on a non-finite X^{n+1}
  const int *layer;   // 2-D batches: layer of each point (null: layer 0)
  const double *dt_layer;  // 2-D batches: time step of each layer (null: dt)
  int64_t np;
  Grid g;
  double inv_h, dt;
  int evolve, first;
};

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_interp(InterpArgs<T, DIM> a) {
  using C = T;
  // Four lanes per (point, component): lane q takes stencil column t0 = q of
  // every row (16 rows in 3-D, 4 in 2-D), so the four lanes of a point read
  // four consecutive cells of a row together -- one wave load touches 16
  // rows, not the 64 it touched when each lane walked a whole plane (the
  // gathers were bound by the cache lines per load: 253 -> 177 us for the
  // 933,888-point cylinder) -- and the four partial sums meet through two
  // lane exchanges.
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t k = gid >> 2;
  const int q = (int)(gid & 3);  // the stencil column t0 this lane reads
  const int c = blockIdx.y;
  if (k >= a.np) return;  // all four lanes of a point leave together
  const int64_t lay = (DIM == 2 && a.layer) ? a.layer[k] : 0;
  const int32_t nn[3] = {a.g.n0, a.g.n1, a.g.n2};
  C w[3][4];
  int b[3];
  for (int ax = 0; ax < DIM; ax++)
    b[ax] = axis_stencil<C>(a.X[ax * a.np + k], a.inv_h, ax == c ? 0.0 : 0.5,
                            nn[ax], w[ax]);
  const T *__restrict__ uc = a.u[c];
  int64_t ii = b[0] + q;  // b[0] < n and n >= 4: one wrap at most
  ii -= ii >= nn[0] ? nn[0] : 0;
  C acc = 0;
  if (DIM == 3) {
#pragma unroll
    for (int t2 = 0; t2 < 4; t2++) {
      int64_t kk = b[2] + t2;
      kk -= kk >= nn[2] ? nn[2] : 0;
      C acc1 = 0;
#pragma unroll
      for (int t1 = 0; t1 < 4; t1++) {
        int64_t jj = b[1] + t1;
        jj -= jj >= nn[1] ? nn[1] : 0;
        acc1 += (C)uc[(kk * nn[1] + jj) * nn[0] + ii] * w[1][t1];
      }
      acc += acc1 * w[2][t2];
    }
  } else {
#pragma unroll
    for (int t1 = 0; t1 < 4; t1++) {
      int64_t jj = b[1] + t1;
      jj -= jj >= nn[1] ? nn[1] : 0;
      acc += (C)uc[(lay * nn[1] + jj) * nn[0] + ii] * w[1][t1];
    }
  }
  acc *= q == 0 ? w[0][0] : q == 1 ? w[0][1] : q == 2 ? w[0][2] : w[0][3];
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  if (q != 0) return;
  const double U = (double)acc;
  const int64_t o = c * a.np + k;
  if (!a.evolve) {
    a.U[o] = U;
    return;
  }
  const double x = a.X[o];
  const double dt = a.dt_layer ? a.dt_layer[lay] : a.dt;
  const double xn1 = a.first ? x + dt * U : x + dt * (1.5 * U - 0.5 * a.U[o]);
  a.U[o] = U;
  a.Xn1[o] = xn1;
  a.Xh[o] = 0.5 * (xn1 + x);
  if (!isfinite(xn1)) *a.flag = 1;
}

// ----------------------------------------------------- Lagrangian: Step 2a --

// One thread per point: gather the link forces at X^{n+1/2} over the point's
// incident links (CSR by point), F_k = sum kappa (X_l - X_k)(1 - l0/|X_l - X_k|),
// plus a tethered point's pull kappa_t (Y_k - X_k) towards its fixed target.
// X_l - X_k is the nearest periodic image (the box is periodic and a fiber
// may close through its periodic copy, as the axial fibers of the cylinder
// of Sec. "Cylindrical Shell in 3D" do).  When Xn1 != null also commit
// X <- X^{n+1} for the point.
template <int DIM>
struct ForceArgs {
  const int32_t *ptr, *nbr;
  const double *kap, *l0;
  const double *Xh;
  double *F;
  const double *Xn1;
  double *X;
  int64_t np;
  double box[DIM];  // periodic box length per axis
  const double *tk, *ty;  // tethers: stiffness [np], target [DIM][np] (null: none)
};

template <int DIM>
__device__ __forceinline__ void force_point(const ForceArgs<DIM> &a, int64_t k) {
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
      d[c] -= a.box[c] * round(d[c] / a.box[c]);
      len2 += d[c] * d[c];
    }
    double t = a.kap[e];
    const double r0 = a.l0[e];
    if (r0 != 0.0) t *= 1.0 - r0 / sqrt(len2);
    for (int c = 0; c < DIM; c++) f[c] += t * d[c];
  }
  if (a.tk) {  // tether: kappa_t (Y_k - X_k), nearest image
    const double t = a.tk[k];
    for (int c = 0; c < DIM; c++) {
      double d = a.ty[c * a.np + k] - xk[c];
      d -= a.box[c] * round(d / a.box[c]);
      f[c] += t * d;
    }
  }
  for (int c = 0; c < DIM; c++) a.F[c * a.np + k] = f[c];
  if (a.Xn1)
    for (int c = 0; c < DIM; c++) a.X[c * a.np + k] = a.Xn1[c * a.np + k];
}

template <int DIM>
__global__ void __launch_bounds__(256) k_force(ForceArgs<DIM> a) {
  force_point<DIM>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ----------------------------------------------------- Lagrangian: Step 2b --
//
// Spreading is an owner-computes gather over cubic tiles of TS cells:
//  1. k_bin, the scan of the tile counts (k_scan_*) and scatter_point
//     counting-sort the points by the tile
//     of their anchor cell a = floor(X/h - 1/2) - 1 (per axis).  Every MAC
//     component's 4-point stencil starts at a or a + 1, so a point touches
//     cells a .. a+4 along each axis.
//  2. touch_tile lists the tiles some stencil reaches (and flags them for
//     the explicit step), in the same launch as scatter_point
//     (k_scatter_touch); k_spread_tiles then collects, for each listed tile,
//     every (point, stencil row) of the tiles whose anchors lie within 4
//     cells below it that lands in the tile, accumulates in LDS and writes
//     the tile's cells (store mode: f = sum; add mode: f += sum).  No
//     global atomics on f; unlisted tiles are flagged empty, never read.

constexpr int TS = 8;

struct TileGrid {
  int32_t nt[3];    // tiles per axis
  int64_t ntiles;
};

__device__ __forceinline__ int anchor_cell(double x, double inv_h, int n) {
  double xi = x * inv_h - 0.5;
  if (!(fabs(xi) < 1e7)) xi = 0.0;  // non-finite positions land in cell 0
  return wrap_cell((int)floor(xi) - 1, n);
}

// (2-D batches: the third tile index is the point's layer.)  The ranks are
// taken per wave: lanes that fall in the same tile (neighbouring points
// usually do) share one atomic on its counter and number themselves in lane
// order, so a dense structure does not queue its points on one address.
// (every lane of the wave calls it, for the ballots)
template <int DIM>
__device__ __forceinline__ void bin_point(const double *X, const int *layer, int64_t np, Grid g,
                                          TileGrid tg, double inv_h, int *count, int *tile_of,
                                          int *rank_of, int64_t k) {
  const bool valid = k < np;
  const int32_t nn[3] = {g.n0, g.n1, g.n2};
  int t = -1;
  if (valid) {
    int64_t tt = 0, mul = 1;
    for (int ax = 0; ax < DIM; ax++) {
      tt += (anchor_cell(X[ax * np + k], inv_h, nn[ax]) / TS) * mul;
      mul *= tg.nt[ax];
    }
    if (DIM == 2 && layer) tt += (int64_t)layer[k] * mul;
    t = (int)tt;
  }
  const int lane = (int)__lane_id();
  uint64_t todo = __ballot(valid);
  int within = 0, leader_of = lane, ntile = 0;
  while (todo) {  // one pass per distinct tile among the wave's points
    const int leader = __builtin_ctzll(todo);
    const int tl = __shfl(t, leader);
    const uint64_t same = __ballot(valid && t == tl);
    if (valid && t == tl) {
      within = __popcll(same & ((1ull << lane) - 1ull));
      leader_of = leader;
    }
    if (lane == leader) ntile = __popcll(same);
    todo &= ~same;
  }
  // the leaders' atomics all in flight at once (one round trip, not one per
  // distinct tile), then every lane reads its leader's base
  int base = 0;
  if (ntile) base = atomicAdd(&count[t], ntile);
  base = __shfl(base, leader_of);
  if (valid) {
    tile_of[k] = t;
    rank_of[k] = base + within;
  }
}

template <int DIM>
__global__ void __launch_bounds__(256) k_bin(const double *X, const int *layer, int64_t np,
                                              Grid g, TileGrid tg, double inv_h, int *count,
                                              int *tile_of, int *rank_of) {
  bin_point<DIM>(X, layer, np, g, tg, inv_h, count, tile_of, rank_of,
                 (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Steps 2a and the first pass of 2b in one launch, one thread per point: the
// link force at X^{n+1/2} (committing X^{n+1}), then the point's spreading
// tile and rank, from the same X^{n+1/2}.  (The force writes F and X; the
// binning reads only X^{n+1/2}.)
template <int DIM>
__global__ void __launch_bounds__(256) k_force_bin(ForceArgs<DIM> a, const int *layer, Grid g,
                                                    TileGrid tg, double inv_h, int *count,
                                                    int *tile_of, int *rank_of) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  force_point<DIM>(a, k);
  bin_point<DIM>(a.Xh, layer, a.np, g, tg, inv_h, count, tile_of, rank_of, k);
}

// Exclusive scan of the per-tile counts into start[0..ntiles] in three
// passes over blocks of SCAN_TILE counts (4 per thread): block sums, a scan
// of the block sums, then each block's own scan; the counts are cleared for
// the next step.
constexpr int SCAN_TILE = 1024;

__device__ __forceinline__ int block_exclusive_scan256(int v, int *sh, int &total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int add = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  total = sh[255];
  const int incl = sh[tid];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(256) k_scan_sums(const int *count, int *bsum, int64_t ntiles) {
  __shared__ int sh[256];
  const int64_t b = (int64_t)blockIdx.x * SCAN_TILE + 4 * threadIdx.x;
  int v = 0;
  for (int q = 0; q < 4; q++)
    if (b + q < ntiles) v += count[b + q];
  int total;
  block_exclusive_scan256(v, sh, total);
  if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) k_scan_bsums(int *bsum, int nb, int *nlist) {
  __shared__ int sh[256];
  if (threadIdx.x == 0) *nlist = 0;
  const int per = (nb + 255) / 256;
  const int b = threadIdx.x * per;
  int v = 0;
  for (int q = 0; q < per; q++)
    if (b + q < nb) v += bsum[b + q];
  int total;
  int run = block_exclusive_scan256(v, sh, total);
  for (int q = 0; q < per; q++)
    if (b + q < nb) {
      const int c = bsum[b + q];
      bsum[b + q] = run;
      run += c;
    }
}

__global__ void __launch_bounds__(256) k_scan_write(int *count, int *start, const int *bsum,
                                                    int64_t ntiles) {
  __shared__ int sh[256];
  const int64_t b = (int64_t)blockIdx.x * SCAN_TILE + 4 * threadIdx.x;
  int c[4], v = 0;
  for (int q = 0; q < 4; q++) {
    c[q] = b + q < ntiles ? count[b + q] : 0;
    v += c[q];
  }
  int total;
  int run = block_exclusive_scan256(v, sh, total) + bsum[blockIdx.x];
  for (int q = 0; q < 4; q++)
    if (b + q < ntiles) {
      start[b + q] = run;
      run += c[q];
      count[b + q] = 0;
    }
  if (b < ntiles && b + 4 >= ntiles) start[ntiles] = run;
}

// The same scan in one launch of one workgroup (1024 threads) when there are
// at most SCAN_ONE_MAX tiles (all the grids of the step's workloads): chunks
// of 4096 counts (one 16-byte load per thread, eight chunks' loads in flight
// at a time) are scanned one after another across the workgroup -- a lane
// scan, the wave totals through LDS -- on top of the running total of the
// chunks before.  Also clears the touched-tile count (as k_scan_bsums does).
constexpr int SCAN_ONE_THREADS = 1024;
constexpr int64_t SCAN_ONE_MAX = 65536;

__global__ void __launch_bounds__(1024) k_scan_one(int *count, int *start, int64_t ntiles,
                                                   int *nlist) {
  __shared__ int wsum[SCAN_ONE_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nchunk = (int)((ntiles + 4095) / 4096);
  if (tid == 0) *nlist = 0;
  int total = 0;  // counts of the chunks before (the same in every thread)
  for (int k0 = 0; k0 < nchunk; k0 += 8) {
    int4 v[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
      const int64_t i = ((int64_t)(k0 + k) * SCAN_ONE_THREADS + tid) * 4;
      if (i + 3 < ntiles) {
        v[k] = *reinterpret_cast<const int4 *>(count + i);
      } else {
        v[k].x = i < ntiles ? count[i] : 0;
        v[k].y = i + 1 < ntiles ? count[i + 1] : 0;
        v[k].z = i + 2 < ntiles ? count[i + 2] : 0;
        v[k].w = 0;
      }
    }
#pragma unroll
    for (int k = 0; k < 8; k++) {
      if (k0 + k >= nchunk) break;  // uniform
      const int s4 = v[k].x + v[k].y + v[k].z + v[k].w;
      int incl = s4;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
      }
      if (lane == 63) wsum[wv] = incl;
      __syncthreads();
      int before = 0, chunk = 0;
#pragma unroll
      for (int w = 0; w < SCAN_ONE_THREADS / 64; w++) {
        const int t = wsum[w];
        before += w < wv ? t : 0;
        chunk += t;
      }
      __syncthreads();  // wsum is rewritten by the next chunk
      const int64_t i = ((int64_t)(k0 + k) * SCAN_ONE_THREADS + tid) * 4;
      int4 st;
      st.x = total + before + incl - s4;
      st.y = st.x + v[k].x;
      st.z = st.y + v[k].y;
      st.w = st.z + v[k].z;
      if (i + 3 < ntiles) {
        *reinterpret_cast<int4 *>(start + i) = st;
        *reinterpret_cast<int4 *>(count + i) = make_int4(0, 0, 0, 0);
      } else {
        if (i < ntiles) start[i] = st.x, count[i] = 0;
        if (i + 1 < ntiles) start[i + 1] = st.y, count[i + 1] = 0;
        if (i + 2 < ntiles) start[i + 2] = st.z, count[i + 2] = 0;
      }
      total += chunk;
    }
  }
  if (tid == 0) start[ntiles] = total;
}

// Place every point at its sorted slot: its position (FP64) and, per
// component, the spread value F_c w / h^d.  The spreading kernels compute
// each stencil from the position where they use it (three square roots per
// point and component, hidden under the LDS atomics): tables of start cells
// and weights per point (30 values in 3-D) cost more to write and read back
// than the arithmetic they save -- the 933,888-point cylinder's sort pass
// wrote 132 bytes per point for them.  The weights come out bitwise the
// same, computed in the grid precision from the same FP64 coordinate.
template <typename T>
struct Sorted {
  double *x;  // [ax * np + slot]
  T *val;     // [c * np + slot]
};

template <typename T, int DIM>
__device__ __forceinline__ void scatter_point(int64_t i, const int *tile_of, const int *rank_of,
                                              const int *start, const int *point_of,
                                              const double *X, const double *F, const double *w,
                                              Sorted<T> st, double inv_hd, int64_t np) {
  if (i >= np) return;
  // i is a point (slot start[tile] + rank) or, with point_of (the
  // deterministic order), a slot whose point point_of[i] is
  const int64_t k = point_of ? point_of[i] : i;
  const int64_t d = point_of ? i : start[tile_of[k]] + rank_of[k];
  for (int ax = 0; ax < DIM; ax++) st.x[ax * np + d] = X[ax * np + k];
  const double wk = w[k] * inv_hd;
  for (int c = 0; c < DIM; c++) st.val[c * np + d] = (T)(F[c * np + k] * wk);
}

// Tiles whose cells lie within 4 cells above an anchor tile, per axis: the
// tiles holding the cells lo-4 .. hi-1 (cyclic), at most 3 distinct.
__device__ __forceinline__ int source_tiles(int lo, int hi, int n, int list[3]) {
  int len = 0;
  for (int cell = lo - 4; cell < hi; cell++) {
    const int tt = wrap_cell(cell, n) / TS;
    bool seen = false;
    for (int q = 0; q < len; q++) seen |= list[q] == tt;
    if (!seen && len < 3) list[len++] = tt;
  }
  return len;
}

// One thread per tile: does any point's stencil reach the tile?  Touched
// tiles are appended to `list` (order arbitrary) and, in store mode, every
// tile's flag records whether f holds force there.  A wave reserves the
// list slots of all its touched tiles with one atomic (consecutive slots in
// lane order) instead of one atomic per tile on the shared counter.
// (t: the tile of this thread; every lane of the wave calls it, for the
// ballot)
template <int DIM>
__device__ __forceinline__ void touch_tile(int t, const int *start, int *flag, int *list,
                                           int *nlist, Grid g, TileGrid tg) {
  // tile counts stay below 2^31 (at most (1024/8)^3 tiles, or 128^2 tiles
  // times 65535 layers in 2-D), so the index arithmetic is 32-bit
  bool hit = false;
  if (t < tg.ntiles) {  // every lane stays for the ballot below
    const int32_t nn[3] = {g.n0, g.n1, g.n2};
    const int nt0 = tg.nt[0], nt1 = tg.nt[1];
    const int tc[3] = {t % nt0, (t / nt0) % nt1, t / (nt0 * nt1)};
    int lst[3][3], len[3];
    for (int ax = 0; ax < 3; ax++) {
      if (ax >= DIM) {
        lst[ax][0] = tc[ax];  // 2-D: the tile's own layer
        len[ax] = 1;
      } else {
        len[ax] = source_tiles(tc[ax] * TS, min(nn[ax], tc[ax] * TS + TS), nn[ax], lst[ax]);
      }
      for (int q = len[ax]; q < 3; q++) lst[ax][q] = lst[ax][0];  // valid fillers
    }
    // fixed trip counts, every count read issued up front (the fillers read
    // real entries and are masked out), so the reads overlap instead of
    // waiting one after another
    int total = 0;
#pragma unroll
    for (int i2 = 0; i2 < (DIM == 3 ? 3 : 1); i2++)
#pragma unroll
      for (int i1 = 0; i1 < 3; i1++)
#pragma unroll
        for (int i0 = 0; i0 < 3; i0++) {
          const int tt = lst[0][i0] + nt0 * (lst[1][i1] + nt1 * lst[2][i2]);
          const int cnt = start[tt + 1] - start[tt];
          total += (i0 < len[0] && i1 < len[1] && i2 < len[2]) ? cnt : 0;
        }
    if (flag) flag[t] = total > 0;
    hit = total > 0;
  }
  const uint64_t m = __ballot(hit);
  if (m == 0) return;
  const int lane = (int)__lane_id();
  const int leader = __builtin_ctzll(m);
  int base = 0;
  if (lane == leader) base = atomicAdd(nlist, __popcll(m));
  base = __shfl(base, leader);
  if (hit) list[base + __popcll(m & ((1ull << lane) - 1ull))] = (int)t;
}

// One launch for the two passes that need only the tile starts: workgroups
// [0, pblocks) place the points (scatter_point), the rest list the touched
// tiles (touch_tile).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_scatter_touch(const int *tile_of, const int *rank_of,
                                                        const int *start, const int *point_of,
                                                        const double *X, const double *F,
                                                        const double *w, Sorted<T> st, Grid g,
                                                        double inv_hd, int64_t np,
                                                        int pblocks, int *flag, int *list,
                                                        int *nlist, TileGrid tg) {
  if ((int)blockIdx.x < pblocks)
    scatter_point<T, DIM>((int64_t)blockIdx.x * blockDim.x + threadIdx.x, tile_of, rank_of, start,
                          point_of, X, F, w, st, inv_hd, np);
  else
    touch_tile<DIM>((int)((blockIdx.x - pblocks) * blockDim.x + threadIdx.x), start, flag, list,
                    nlist, g, tg);
}

// Deterministic order (IB_FLAG_DETERMINISTIC_SPREAD).  The ranks k_bin
// hands out within a tile depend on the order in which waves reach the tile
// counters; here every point is first placed at its slot (point_of), then
// each tile's points are put in point-index order (one thread per tile,
// insertion sort of the tile's few points), so the sorted order -- and the
// order in which k_spread_det adds them -- no longer depends on scheduling.
__global__ void __launch_bounds__(256) k_place(const int *tile_of, const int *rank_of,
                                               const int *start, int *point_of, int64_t np) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < np) point_of[start[tile_of[k]] + rank_of[k]] = (int)k;
}

__global__ void __launch_bounds__(256) k_order_tiles(const int *start, int *point_of,
                                                     int64_t ntiles) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ntiles) return;
  const int b = start[t], e = start[t + 1];
  for (int i = b + 1; i < e; i++) {
    const int v = point_of[i];
    int j = i - 1;
    while (j >= b && point_of[j] > v) {
      point_of[j + 1] = point_of[j];
      j--;
    }
    point_of[j + 1] = v;
  }
}

template <typename T, int DIM>
struct SpreadArgs {
  Sorted<T> st;  // points in sorted order
  double inv_h;
  T *f[3];
  const int *start, *list, *nlist;
  int64_t np;
  Grid g;
  TileGrid tg;
};

// Workgroups loop over the touched tiles (a bounded loop: at most ntiles
// entries).  For each tile: gather (point, stencil row) items of the source
// tiles into LDS, then write the tile's cells (f = sum, or f += sum).  The
// LDS sums are FP64 (A) also for an FP32 grid: gfx950's LDS takes FP64 atomic
// adds at about twice the rate of FP32 ones (measured: 711 vs 1271 us for the
// 933,888-point cylinder at 256^3), and the sum is rounded to FP32 once.
//
// The LDS sums are laid out with padded strides: rows of TS + 1 slots,
// planes of TS (TS + 1), and each component's array offset by 5 slots more.
// With x fastest and unpadded rows of 8 doubles, cells that differ in y or
// z fall on the same two banks; the points of a dense sheet handled by one
// wave differ exactly there (a wave takes neighbouring points along the
// sheet), so their atomics queued on one bank.  Padded, neighbours in y and
// z and the three components land on different banks.
constexpr int SP_ROW = TS + 1;                  // slot stride of a tile row
constexpr int SP_PLANE = TS * SP_ROW;           // slot stride of a tile plane
template <int DIM>
constexpr int sp_comp() { return (DIM == 3 ? TS * SP_PLANE : SP_PLANE) + 5; }

template <typename T, int DIM, bool ADD, int NT = 256, typename A = double>
__global__ void __launch_bounds__(NT) k_spread_tiles(SpreadArgs<T, DIM> a) {
  using C = T;
  constexpr int CELLS = DIM == 3 ? TS * TS * TS : TS * TS;
  constexpr int CS = sp_comp<DIM>();
  __shared__ A acc[DIM * CS];
  __shared__ int c_start[27], c_pref[28], s_list[3][3], s_len[3], s_cnt[27];
  const int32_t nn[3] = {a.g.n0, a.g.n1, a.g.n2};
  int ntodo = *a.nlist;
  ntodo = ntodo < a.tg.ntiles ? ntodo : (int)a.tg.ntiles;
  for (int e = blockIdx.x; e < ntodo; e += gridDim.x) {
    const int64_t t = a.list[e];
    const int tc[3] = {(int)(t % a.tg.nt[0]), (int)((t / a.tg.nt[0]) % a.tg.nt[1]),
                       (int)(t / ((int64_t)a.tg.nt[0] * a.tg.nt[1]))};
    int lo[3], hi[3];
    for (int ax = 0; ax < 3; ax++) {
      lo[ax] = ax < DIM ? tc[ax] * TS : tc[ax];  // 2-D: the tile's layer
      hi[ax] = ax < DIM ? min(nn[ax], lo[ax] + TS) : lo[ax] + 1;
    }
    if (threadIdx.x < 3) {
      const int ax = threadIdx.x;
      if (ax >= DIM) {
        s_list[ax][0] = tc[ax];
        s_len[ax] = 1;
      } else {
        int l3[3];
        const int len = source_tiles(lo[ax], hi[ax], nn[ax], l3);
        for (int q = 0; q < len; q++) s_list[ax][q] = l3[q];
        s_len[ax] = len;
      }
    }
    for (int i = threadIdx.x; i < DIM * CS; i += blockDim.x) acc[i] = A(0);
    __syncthreads();
    const int ncomb = s_len[0] * s_len[1] * s_len[2];
    if (threadIdx.x < ncomb) {
      const int m = threadIdx.x;
      const int i0 = m % s_len[0], i1 = (m / s_len[0]) % s_len[1], i2 = m / (s_len[0] * s_len[1]);
      const int64_t tt = s_list[0][i0] + (int64_t)a.tg.nt[0] *
                                             (s_list[1][i1] + (int64_t)a.tg.nt[1] * s_list[2][i2]);
      const int s0 = a.start[tt];
      c_start[m] = s0;
      s_cnt[m] = a.start[tt + 1] - s0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int pref = 0;
      for (int m = 0; m < ncomb; m++) {
        c_pref[m] = pref;
        pref += s_cnt[m];
      }
      c_pref[ncomb] = pref;
    }
    __syncthreads();
    // one thread per candidate point; only the stencil rows and columns that
    // fall inside the tile are visited
    const int npts = c_pref[ncomb];
    const int64_t np = a.np;
    // one thread per (candidate point, component): the DIM-fold parallelism
    // hides more of the atomics' latency than one thread walking all
    // components (3-D: 754 -> 614 us for the 933,888-point cylinder, 73 ->
    // 66 us for the 65,536-point shell)
    constexpr int PER = DIM;
    // 256-thread workgroups deal the items of a block to lanes transposed:
    // lane l of wave w takes item 4 l + w, so one wave's atomics come from
    // points four items apart instead of neighbours along a sheet (whose
    // stencils overlap, and whose atomics on one address queue).  The dense
    // 1024-thread kernel keeps the items in order (transposed, the 128^3
    // shell of the closure's coarse step spread slower).
    const int perm = NT == 256 ? (int)(threadIdx.x % 64) * 4 + (int)(threadIdx.x / 64)
                               : (int)threadIdx.x;
    for (int base = 0; base < npts * PER; base += NT) {
      const int it = base + perm;
      if (it >= npts * PER) continue;
      const int pi = it / PER;
      int slot = 0;
      while (c_pref[slot + 1] <= pi) slot++;
      const int64_t k = c_start[slot] + (pi - c_pref[slot]);
      const int c_lo = PER == 1 ? 0 : it - pi * PER, c_hi = PER == 1 ? DIM : c_lo + 1;
      for (int c = c_lo; c < c_hi; c++) {
        // in-tile coordinate of each stencil offset t = 0..3 per axis, -1
        // where (b + t) mod n falls outside the tile.  The in-tile offsets
        // need not be contiguous: on an axis of at most 10 cells tile 0 can
        // hold cells from both sides of the periodic wrap (n = 9, b = 7:
        // cells 7, 8, 0, 1, of which 7, 0, 1 lie in tile 0).
        int loc[3][4];
        bool any = true;
        // component c's stencil along each axis, from the sorted position
        C wx[4], wy[4], wz[4] = {C(1), C(0), C(0), C(0)};
        int b3[3] = {0, 0, 0};
        b3[0] = axis_stencil<C>(a.st.x[k], a.inv_h, c == 0 ? 0.0 : 0.5, nn[0], wx);
        b3[1] = axis_stencil<C>(a.st.x[np + k], a.inv_h, c == 1 ? 0.0 : 0.5, nn[1], wy);
        if (DIM == 3) b3[2] = axis_stencil<C>(a.st.x[2 * np + k], a.inv_h, c == 2 ? 0.0 : 0.5, nn[2], wz);
#pragma unroll
        for (int ax = 0; ax < 3; ax++) {
          bool hit = false;
          const int b0 = b3[ax];
#pragma unroll
          for (int t = 0; t < 4; t++) {
            if (ax >= DIM) {  // 2-D: the tile's own layer, one offset
              loc[ax][t] = t == 0 ? 0 : -1;
              continue;
            }
            int cell = b0 + t;  // b0 < n and n >= 4: one wrap at most
            cell -= cell >= nn[ax] ? nn[ax] : 0;
            const bool in = cell >= lo[ax] && cell < hi[ax];
            loc[ax][t] = in ? cell - lo[ax] : -1;
            hit |= in;
          }
          any &= ax >= DIM || hit;
        }
        if (!any) continue;
        const C val = a.st.val[c * np + k];
#pragma unroll
        for (int t2 = 0; t2 < (DIM == 3 ? 4 : 1); t2++) {
          const int lz = loc[2][t2];
          if (lz < 0) continue;
#pragma unroll
          for (int t1 = 0; t1 < 4; t1++) {
            const int ly = loc[1][t1];
            if (ly < 0) continue;
            const C rw = val * wz[t2] * wy[t1];
            const int lrow = c * CS + lz * SP_PLANE + ly * SP_ROW;
#pragma unroll
            for (int t0 = 0; t0 < 4; t0++)
              if (loc[0][t0] >= 0) atomicAdd(&acc[lrow + loc[0][t0]], (A)(rw * wx[t0]));
          }
        }
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < CELLS; i += blockDim.x) {
      const int li = i % TS, lj = (i / TS) % TS, lk = DIM == 3 ? i / (TS * TS) : 0;
      const int gi = lo[0] + li, gj = lo[1] + lj, gk = lo[2] + lk;
      if (gi >= hi[0] || gj >= hi[1] || gk >= hi[2]) continue;
      const int64_t idx = gi + (int64_t)nn[0] * (gj + (int64_t)nn[1] * gk);
      const int sl = lk * SP_PLANE + lj * SP_ROW + li;
      for (int c = 0; c < DIM; c++) {
        if (ADD) a.f[c][idx] = (T)((A)a.f[c][idx] + acc[c * CS + sl]);
        else a.f[c][idx] = (T)acc[c * CS + sl];
      }
    }
    __syncthreads();
  }
}

// Deterministic spreading: the same tiles and candidates as k_spread_tiles,
// but no atomics -- each thread owns cells of the tile and adds, in the fixed
// candidate order (source tiles in a fixed order, points in slot order), the
// stencil weight every candidate puts on its cell, in FP64 registers.  Every
// cell's sum is then formed in one order, whatever the scheduling.  (Each
// cell visits every candidate: a mode for verification and bitwise restarts,
// not for speed.)
template <typename T, int DIM, bool ADD>
__global__ void __launch_bounds__(256) k_spread_det(SpreadArgs<T, DIM> a) {
  using C = T;
  constexpr int CELLS = DIM == 3 ? TS * TS * TS : TS * TS;
  constexpr int PER = (CELLS + 255) / 256;
  __shared__ int c_start[27], c_pref[28], s_list[3][3], s_len[3], s_cnt[27];
  const int32_t nn[3] = {a.g.n0, a.g.n1, a.g.n2};
  int ntodo = *a.nlist;
  ntodo = ntodo < a.tg.ntiles ? ntodo : (int)a.tg.ntiles;
  for (int e = blockIdx.x; e < ntodo; e += gridDim.x) {
    const int64_t t = a.list[e];
    const int tc[3] = {(int)(t % a.tg.nt[0]), (int)((t / a.tg.nt[0]) % a.tg.nt[1]),
                       (int)(t / ((int64_t)a.tg.nt[0] * a.tg.nt[1]))};
    int lo[3], hi[3];
    for (int ax = 0; ax < 3; ax++) {
      lo[ax] = ax < DIM ? tc[ax] * TS : tc[ax];
      hi[ax] = ax < DIM ? min(nn[ax], lo[ax] + TS) : lo[ax] + 1;
    }
    if (threadIdx.x < 3) {
      const int ax = threadIdx.x;
      if (ax >= DIM) {
        s_list[ax][0] = tc[ax];
        s_len[ax] = 1;
      } else {
        int l3[3];
        const int len = source_tiles(lo[ax], hi[ax], nn[ax], l3);
        for (int q = 0; q < len; q++) s_list[ax][q] = l3[q];
        s_len[ax] = len;
      }
    }
    __syncthreads();
    const int ncomb = s_len[0] * s_len[1] * s_len[2];
    if (threadIdx.x < ncomb) {
      const int m = threadIdx.x;
      const int i0 = m % s_len[0], i1 = (m / s_len[0]) % s_len[1], i2 = m / (s_len[0] * s_len[1]);
      const int64_t tt = s_list[0][i0] + (int64_t)a.tg.nt[0] *
                                             (s_list[1][i1] + (int64_t)a.tg.nt[1] * s_list[2][i2]);
      const int s0 = a.start[tt];
      c_start[m] = s0;
      s_cnt[m] = a.start[tt + 1] - s0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int pref = 0;
      for (int m = 0; m < ncomb; m++) {
        c_pref[m] = pref;
        pref += s_cnt[m];
      }
      c_pref[ncomb] = pref;
    }
    __syncthreads();
    const int npts = c_pref[ncomb];
    const int64_t np = a.np;
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const int i = threadIdx.x + q * 256;
      if (i >= CELLS) break;
      const int g3[3] = {lo[0] + i % TS, lo[1] + (i / TS) % TS, DIM == 3 ? lo[2] + i / (TS * TS) : lo[2]};
      if (g3[0] >= hi[0] || g3[1] >= hi[1] || g3[2] >= hi[2]) continue;
      double acc[DIM];
      for (int c = 0; c < DIM; c++) acc[c] = 0.0;
      int slot = 0;
      for (int pi = 0; pi < npts; pi++) {
        while (c_pref[slot + 1] <= pi) slot++;
        const int64_t k = c_start[slot] + (pi - c_pref[slot]);
        for (int c = 0; c < DIM; c++) {
          // offset of this cell in the point's stencil along each axis
          int off[3] = {0, 0, 0};
          C wt[3][4];
          bool in = true;
          for (int ax = 0; ax < DIM; ax++) {
            const int b0 = axis_stencil<C>(a.st.x[ax * np + k], a.inv_h, ax == c ? 0.0 : 0.5,
                                           nn[ax], wt[ax]);
            int o = g3[ax] - b0;
            o += o < 0 ? nn[ax] : 0;  // base < n, cell < n: one wrap at most
            in &= o < 4;
            off[ax] = in ? o : 0;
          }
          if (!in) continue;
          // the product in k_spread_tiles' order: (value z-weight) y-weight,
          // then times the x-weight
          C rw = a.st.val[c * np + k];
          if (DIM == 3) rw = rw * wt[2][off[2]];
          rw = rw * wt[1][off[1]];
          acc[c] += (double)(rw * wt[0][off[0]]);
        }
      }
      const int64_t idx = g3[0] + (int64_t)nn[0] * (g3[1] + (int64_t)nn[1] * g3[2]);
      for (int c = 0; c < DIM; c++) {
        if (ADD) a.f[c][idx] = (T)((double)a.f[c][idx] + acc[c]);
        else a.f[c][idx] = (T)acc[c];
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------ Eulerian: Steps 3a-3b fused --

// Dense copy of the force density spread in the last step: f where the
// tile was flagged as holding force, 0 elsewhere (the spreading never writes
// unflagged tiles).
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_force_dense(const T *f0, const T *f1, const T *f2,
                                                      const int *flag, Grid g, TileGrid tg,
                                                      T *o0, T *o1, T *o2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.ncell) return;
  const int i = (int)(idx % g.n0);
  const int j = (int)((idx / g.n0) % g.n1);
  const int k = (int)(idx / ((int64_t)g.n0 * g.n1));
  const int64_t tile =
      i / TS + (int64_t)tg.nt[0] * (j / TS + (int64_t)tg.nt[1] * (DIM == 3 ? k / TS : k));
  const bool forced = flag[tile] != 0;
  o0[idx] = forced ? f0[idx] : T(0);
  o1[idx] = forced ? f1[idx] : T(0);
  if (DIM == 3) o2[idx] = forced ? f2[idx] : T(0);
}

// One thread per cell.  For each component c at its face:
//   N_c  = skew advection (Morinishi 2nd-order staggered: 1/2 divergence form
//          + 1/2 advective form),
//   Nh   = 3/2 N_c - 1/2 N_c^{n-1}   (N_c alone at n = 0),
//   d*_c = dt ( -Nh + (mu Lap u_c - G_c p* + f_c)/rho ),  p* = p + psi (FP64),
// and stores d*_c (the delta-form right-hand side of the first sweep) and
// N_c into nl (for the next step).  f_c is read only in tiles the spreading
// flagged as holding force (zero elsewhere).
template <typename T, int DIM, typename V = T>
struct ExplicitArgs {
  const V *u[3];  // velocity state (V = double under the FP64-state policy)
  T *nl[3];
  const T *f[3];
  T *delta[3];
  const double *p;
  const T *psi;
  const int *flag;  // per spreading tile: 1 if f holds force there
  const double *dt_layer;  // 2-D batches: time step of each layer (null: dt)
  Grid g;
  TileGrid tg;
  double inv_h, inv_h2, dt, mu, inv_rho;
  int first, advect;
  int walls;  // channel: no-slip walls at y = 0 and y = n1 h
  double wall_u[3];  // velocity of the upper wall (tangential components)
  double g_body[3];  // uniform body force density added to f
  int ez;  // planes per workgroup of the 3-D plane-marching kernel
};

template <typename T, int DIM, typename V = T>
__global__ void __launch_bounds__(256) k_explicit(ExplicitArgs<T, DIM, V> a) {
  using C = V;  // arithmetic in the precision of the velocity state
  // blockDim (64, 4): x from blockIdx.x, y from blockIdx.y, the slowest
  // index (z, or the layer of a 2-D batch) from blockIdx.z -- no divisions
  const int64_t n0 = a.g.n0, n1 = a.g.n1, n2 = a.g.n2;
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 4 + threadIdx.y;
  const int64_t k = blockIdx.z;
  if (i >= n0 || j >= n1) return;
  const int64_t idx = i + n0 * (j + n1 * k);
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
  const int64_t tile =
      i / TS + (int64_t)a.tg.nt[0] * (j / TS + (int64_t)a.tg.nt[1] * (DIM == 3 ? k / TS : k));
  const bool forced = a.flag[tile] != 0;
  const C dt = (C)((DIM == 2 && a.dt_layer) ? a.dt_layer[k] : a.dt);
  // channel walls: across y = 0 a tangential component takes the no-slip
  // ghost value -u, across y = n1 h the value 2 U - u of a wall moving with
  // U; v lives on the y faces, whose row 0 is the wall (both walls,
  // periodically) and holds 0, so periodic indexing gives the wall value
  // there and v is not advanced on it
  const bool wlo = a.walls && j == 0, whi = a.walls && j + 1 == n1;
#pragma unroll
  for (int ci = 0; ci < DIM; ci++) {
    if (wlo && ci == 1) {
      a.delta[1][idx] = T(0);
      a.nl[1][idx] = T(0);
      continue;
    }
    const V *__restrict__ ui = a.u[ci];
    const C u0 = (C)ui[idx];
    C dv = 0, ad = 0, lap = 0;
#pragma unroll
    for (int cj = 0; cj < DIM; cj++) {
      C up = (C)ui[idx + dp[cj]], um = (C)ui[idx + dm[cj]];
      if (cj == 1 && ci != 1) {
        if (whi) up = C(2) * (C)a.wall_u[ci] - u0;
        if (wlo) um = -u0;
      }
      lap += up - C(2) * u0 + um;
      if (!a.advect) continue;
      if (cj == ci) {
        const C ap = C(0.5) * (u0 + up), am = C(0.5) * (um + u0);
        dv += ap * ap - am * am;
        ad += C(0.5) * (ap * (up - u0) + am * (u0 - um));
      } else {
        const V *__restrict__ uj = a.u[cj];
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
    const C fc = (forced ? (C)a.f[ci][idx] : C(0)) + (C)a.g_body[ci];
    const C d = dt * (-Nh + ((C)a.mu * lap * (C)a.inv_h2 - gp + fc) * (C)a.inv_rho);
    a.delta[ci][idx] = (T)d;
    a.nl[ci][idx] = (T)N;
  }
}

// ----------------------------------------------- explicit momentum stencil --

// Steps 3a-3b at one cell from three velocity planes held in LDS: returns
// the Laplacian sum and N(u^n) of component ci (skew form, eq:nonlinear).
// at(comp, slot, dx, dy) reads component comp on plane slot (sm: k-1,
// s0: k, sp: k+1) at the in-plane neighbour (dx, dy) of this cell.  The
// z neighbours of a plane are the slots; channel walls replace a tangential
// component's y neighbour across the wall by its no-slip ghost: -u below,
// 2 uw - u above (uw: the upper wall's velocity along ci).
template <typename C, typename At>
__device__ __forceinline__ void momentum_terms(const At &at, int ci, int sm, int s0, int sp,
                                               bool wlo, bool whi, C uw, bool advect, C inv_h,
                                               C &lap, C &N) {
  constexpr int ox[3] = {1, 0, 0}, oy[3] = {0, 1, 0};
  const int slm[3] = {s0, s0, sm}, slp[3] = {s0, s0, sp};
  const C u0 = at(ci, s0, 0, 0);
  C dv = 0, ad = 0;
  lap = 0;
#pragma unroll
  for (int cj = 0; cj < 3; cj++) {
    C up = at(ci, slp[cj], ox[cj], oy[cj]);
    C um = at(ci, slm[cj], -ox[cj], -oy[cj]);
    if (cj == 1 && ci != 1) {  // no-slip ghosts across a channel wall
      if (whi) up = C(2) * uw - u0;
      if (wlo) um = -u0;
    }
    lap += up - C(2) * u0 + um;
    if (!advect) continue;
    if (cj == ci) {
      const C ap = C(0.5) * (u0 + up), am = C(0.5) * (um + u0);
      dv += ap * ap - am * am;
      ad += C(0.5) * (ap * (up - u0) + am * (u0 - um));
    } else {
      // u_cj averaged along ci on the edges at this cell and one up along cj
      const int spm = (ci == 2) ? sm : ((cj == 2) ? sp : s0);
      const C Ua = C(0.5) * (at(cj, slm[ci], -ox[ci], -oy[ci]) + at(cj, s0, 0, 0));
      const C Ub = C(0.5) * (at(cj, spm, ox[cj] - ox[ci], oy[cj] - oy[ci]) +
                             at(cj, slp[cj], ox[cj], oy[cj]));
      dv += Ub * C(0.5) * (u0 + up) - Ua * C(0.5) * (um + u0);
      ad += C(0.5) * (Ub * (up - u0) + Ua * (u0 - um));
    }
  }
  N = C(0.5) * (dv + ad) * inv_h;
}

// 3-D explicit step on a 2.5-D blocking: a workgroup owns an EX x EY tile of
// (x, y) columns and marches a.ez planes along z; the host sizes ez so the
// whole grid is one round of resident workgroups (no tail round), which
// also cuts the prologues and z-halo re-reads.  Three planes of u, v, w
// (tile plus a one-cell halo) and the current plane of p* = p + psi (tile
// plus its -x, -y halo) sit in LDS, so each value is fetched from HBM about
// once instead of once per stencil use.  The loads are software-pipelined:
// while plane k is computed from LDS, plane k+2 of the velocities, plane k+1
// of p* and this cell's N^{n-1} and f are already in flight into registers.
// N^{n-1} is read and N^n written with streaming (non-temporal) hints: neither
// is touched again within the step, so they should not displace delta, which
// the first momentum sweep reads next, from the last-level cache.
// Same arithmetic as k_explicit.
constexpr int EX = 64, EY = 4;
constexpr int EW = EX + 2, EH = EY + 2;  // velocity plane with halo
constexpr int PW = EX + 1, PH = EY + 1;  // p* plane with -x, -y halo
constexpr int ENT = EX * EY;             // threads per workgroup
constexpr int VPT = (EH * EW + ENT - 1) / ENT;  // velocity entries per thread
constexpr int PPT = (PH * PW + ENT - 1) / ENT;  // p* entries per thread

template <typename T, typename V = T>
__global__ void __launch_bounds__(ENT) k_explicit3(ExplicitArgs<T, 3, V> a) {
  using C = V;  // arithmetic in the precision of the velocity state
  __shared__ C U[3][3][EH * EW];
  __shared__ double PS[PH * PW];
  const int n0 = a.g.n0, n1 = a.g.n1, n2 = a.g.n2;
  const int tx = threadIdx.x % EX, ty = threadIdx.x / EX;
  // Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
  // Re-map the 1-D block index so each XCD walks a contiguous run of tiles
  // (x fastest): the halo columns and rows a tile shares with its neighbours
  // are then fetched into one L2.
  const int nbx = n0 / EX, nby = n1 / EY;
  const int nb = gridDim.x;
  const int b = (nb % 8 == 0) ? (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8 : blockIdx.x;
  const int EZ = a.ez;
  const int i0 = (b % nbx) * EX, j0 = ((b / nbx) % nby) * EY, k0 = (b / (nbx * nby)) * EZ;
  const int plane = n0 * n1;  // < 2^31 (checked on the host)
  auto wrap = [](int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); };
  // in-plane offsets of this thread's halo-tile entries and of its own cell,
  // fixed for the whole march; planes only move a wave-uniform base
  int voff[VPT], poff[PPT];
#pragma unroll
  for (int q = 0; q < VPT; q++) {
    const int e = min((int)threadIdx.x + q * ENT, EH * EW - 1);
    voff[q] = wrap(j0 - 1 + e / EW, n1) * n0 + wrap(i0 - 1 + e % EW, n0);
  }
#pragma unroll
  for (int q = 0; q < PPT; q++) {
    const int e = min((int)threadIdx.x + q * ENT, PH * PW - 1);
    poff[q] = wrap(j0 - 1 + e / PW, n1) * n0 + wrap(i0 - 1 + e % PW, n0);
  }
  const int cell = (j0 + ty) * n0 + (i0 + tx);
  // channel walls (as in k_explicit): this thread's row may border one
  const bool wlo = a.walls && j0 + ty == 0, whi = a.walls && j0 + ty == n1 - 1;
  const int tflag_row = (i0 + tx) / TS + a.tg.nt[0] * ((j0 + ty) / TS);
  const int tplane = a.tg.nt[0] * a.tg.nt[1];
  auto pbase = [&](int kk) { return (int64_t)wrap(kk, n2) * plane; };
  // prologue: planes k0-1, k0, k0+1 of the velocities and plane k0 of p*
  for (int sl = 0; sl < 3; sl++) {
    const int64_t pb = pbase(k0 - 1 + sl);
#pragma unroll
    for (int q = 0; q < VPT; q++) {
      const int e = threadIdx.x + q * ENT;
      if (e < EH * EW) {
        U[0][sl][e] = (C)a.u[0][pb + voff[q]];
        U[1][sl][e] = (C)a.u[1][pb + voff[q]];
        U[2][sl][e] = (C)a.u[2][pb + voff[q]];
      }
    }
  }
  {
    const int64_t pb = pbase(k0);
#pragma unroll
    for (int q = 0; q < PPT; q++) {
      const int e = threadIdx.x + q * ENT;
      if (e < PH * PW) PS[e] = a.p[pb + poff[q]] + (double)a.psi[pb + poff[q]];
    }
  }
  const int64_t pbm = pbase(k0 - 1);
  double ps_below = a.p[pbm + cell] + (double)a.psi[pbm + cell];
  const int c = (ty + 1) * EW + (tx + 1);  // this column in a velocity plane
  const int pc = (ty + 1) * PW + (tx + 1);
  // this cell's N^{n-1} and f, one plane ahead of their use
  C nlp[3], fc[3];
  auto cell_terms = [&](int kk, C *nl_out, C *f_out) {
    const int64_t kp = (int64_t)kk * plane;
    const bool forced = a.flag[tflag_row + tplane * (kk / TS)] != 0;
#pragma unroll
    for (int ci = 0; ci < 3; ci++) {
      nl_out[ci] = a.first ? C(0) : (C)__builtin_nontemporal_load(&(a.nl[ci] + kp)[cell]);
      f_out[ci] = (forced ? (C)(a.f[ci] + kp)[cell] : C(0)) + (C)a.g_body[ci];
    }
  };
  cell_terms(k0, nlp, fc);
  __syncthreads();
  for (int kz = 0; kz < EZ && k0 + kz < n2; kz++) {
    const int k = k0 + kz;
    const int sm = kz % 3, s0 = (kz + 1) % 3, sp = (kz + 2) % 3;
    const bool more = kz + 1 < EZ && k + 1 < n2;  // uniform over the workgroup
    // 1. fetch ahead: plane k+2 of u, v, w and plane k+1 of p*
    C vr[3][VPT];
    double pr[PPT];
    if (more) {
      const V *u0p = a.u[0] + pbase(k + 2), *u1p = a.u[1] + pbase(k + 2),
              *u2p = a.u[2] + pbase(k + 2);
#pragma unroll
      for (int q = 0; q < VPT; q++) {
        vr[0][q] = (C)u0p[voff[q]];
        vr[1][q] = (C)u1p[voff[q]];
        vr[2][q] = (C)u2p[voff[q]];
      }
      const double *pp = a.p + pbase(k + 1);
      const T *sp_ = a.psi + pbase(k + 1);
#pragma unroll
      for (int q = 0; q < PPT; q++) pr[q] = pp[poff[q]] + (double)sp_[poff[q]];
    }
    // N^{n-1} and f of plane k+1 (this thread alone reads and writes them)
    C nln[3], fcn[3];
    if (more) cell_terms(k + 1, nln, fcn);
    const int64_t kp = (int64_t)k * plane;
    // 2. compute plane k from LDS
    const double ps0 = PS[pc];
    const double psm[3] = {PS[pc - 1], PS[pc - PW], ps_below};
    auto at = [&](int cp, int s, int dx, int dy) { return U[cp][s][c + dx + dy * EW]; };
#pragma unroll
    for (int ci = 0; ci < 3; ci++) {
      if (wlo && ci == 1) {  // v on the wall face: not advanced
        (a.delta[1] + kp)[cell] = T(0);
        (a.nl[1] + kp)[cell] = T(0);
        continue;
      }
      C lap, N;
      momentum_terms<C>(at, ci, sm, s0, sp, wlo, whi, (C)a.wall_u[ci], a.advect != 0,
                        (C)a.inv_h, lap, N);
      const C gp = (C)((ps0 - psm[ci]) * a.inv_h);
      const C Nh = a.first ? N : C(1.5) * N - C(0.5) * nlp[ci];
      const C d = (C)a.dt * (-Nh + ((C)a.mu * lap * (C)a.inv_h2 - gp + fc[ci]) * (C)a.inv_rho);
      (a.delta[ci] + kp)[cell] = (T)d;
      __builtin_nontemporal_store((T)N, &(a.nl[ci] + kp)[cell]);
    }
    ps_below = ps0;
    // 3. rotate: plane k+2 replaces plane k-1, plane k+1 of p* replaces k
    if (more) {
#pragma unroll
      for (int ci = 0; ci < 3; ci++) nlp[ci] = nln[ci], fc[ci] = fcn[ci];
    }
    __syncthreads();
    if (more) {
#pragma unroll
      for (int q = 0; q < VPT; q++) {
        const int e = threadIdx.x + q * ENT;
        if (e < EH * EW) {
          U[0][sm][e] = vr[0][q];
          U[1][sm][e] = vr[1][q];
          U[2][sm][e] = vr[2][q];
        }
      }
#pragma unroll
      for (int q = 0; q < PPT; q++) {
        const int e = threadIdx.x + q * ENT;
        if (e < PH * PW) PS[e] = pr[q];
      }
    }
    __syncthreads();
  }
}

// D.u at every cell: Step 3e's right-hand side, and the seed div_prev = D.u^0
// (u in the velocity type T, D.u stored in the work type TD).
template <typename T, int DIM, typename TD = T>
__global__ void __launch_bounds__(256) k_divergence(const T *u0, const T *u1,
                                                     const T *u2, TD *out, Grid g,
                                                     double inv_h) {
  // blockDim (64, 4) over (x, y), blockIdx.z the slowest index, as k_explicit
  const int64_t n0 = g.n0, n1 = g.n1, n2 = g.n2;
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t j = (int64_t)blockIdx.y * 4 + threadIdx.y;
  const int64_t k = blockIdx.z;
  if (i >= n0 || j >= n1) return;
  const int64_t idx = i + n0 * (j + n1 * k);
  double s = (double)u0[idx + ((i + 1 == n0) ? -(n0 - 1) : 1)] - (double)u0[idx];
  s += (double)u1[idx + ((j + 1 == n1) ? -(n1 - 1) * n0 : n0)] - (double)u1[idx];
  if (DIM == 3)
    s += (double)u2[idx + ((k + 1 == n2) ? -(n2 - 1) * n0 * n1 : n0 * n1)] -
         (double)u2[idx];
  out[idx] = (TD)(s * inv_h);
}

// Four consecutive cells along x per thread: aligned 16-byte vector loads of
// u, v, w (rows j and j+1, planes k and k+1) and one store of the four
// results, the same sums as k_divergence.  Needs n0 % 4 == 0 and 16-byte
// aligned arrays (checked on the host).  blockDim (64, 4): 256 x-cells of 4
// rows per workgroup.
template <typename T>
__device__ __forceinline__ void load4(const T *p, double v[4]) {
  if constexpr (sizeof(T) == 4) {
    const float4 q = *reinterpret_cast<const float4 *>(p);
    v[0] = q.x, v[1] = q.y, v[2] = q.z, v[3] = q.w;
  } else {
    const double2 q0 = reinterpret_cast<const double2 *>(p)[0];
    const double2 q1 = reinterpret_cast<const double2 *>(p)[1];
    v[0] = q0.x, v[1] = q0.y, v[2] = q1.x, v[3] = q1.y;
  }
}

template <typename T>
__device__ __forceinline__ void store4(T *p, const double v[4]) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4((float)v[0], (float)v[1], (float)v[2], (float)v[3]);
  } else {
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
  }
}

template <typename T, int DIM, typename TD = T>
__global__ void __launch_bounds__(256) k_divergence4(const T *u0, const T *u1,
                                                      const T *u2, TD *out, Grid g,
                                                      double inv_h) {
  const int64_t n0 = g.n0, n1 = g.n1, n2 = g.n2;
  const int64_t i = ((int64_t)blockIdx.x * 64 + threadIdx.x) * 4;
  const int64_t j = (int64_t)blockIdx.y * 4 + threadIdx.y;
  const int64_t k = blockIdx.z;
  if (i >= n0 || j >= n1) return;
  const int64_t idx = i + n0 * (j + n1 * k);
  double a[4], b[4], s[4];
  load4(u0 + idx, a);
  const double next = (double)u0[(i + 4 == n0) ? idx - i : idx + 4];  // x + 4, periodic
  s[0] = a[1] - a[0], s[1] = a[2] - a[1], s[2] = a[3] - a[2], s[3] = next - a[3];
  load4(u1 + idx, a);
  load4(u1 + idx + ((j + 1 == n1) ? -(n1 - 1) * n0 : n0), b);
#pragma unroll
  for (int q = 0; q < 4; q++) s[q] += b[q] - a[q];
  if (DIM == 3) {
    load4(u2 + idx, a);
    load4(u2 + idx + ((k + 1 == n2) ? -(n2 - 1) * n0 * n1 : n0 * n1), b);
#pragma unroll
    for (int q = 0; q < 4; q++) s[q] += b[q] - a[q];
  }
#pragma unroll
  for (int q = 0; q < 4; q++) s[q] *= inv_h;
  store4(out + idx, s);
}

// FP64-state policy: u^{n+1} = u^n + d (the last momentum increment, stored
// in the work precision), accumulated in FP64.
template <typename TD, int DIM>
__global__ void __launch_bounds__(256) k_add_increment(double *u0, double *u1, double *u2,
                                                        const TD *d0, const TD *d1,
                                                        const TD *d2, int64_t ncell) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ncell) return;
  u0[idx] += (double)d0[idx];
  u1[idx] += (double)d1[idx];
  if (DIM == 3) u2[idx] += (double)d2[idx];
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

enum { SW_PLAIN = 0, SW_FINAL = 1, SW_PFINAL = 3 };
// Boundary kinds of a channel's y lines: Dirichlet for a cell-centred unknown
// (ghost -x across the wall), for a face unknown on the wall (element 0, and
// element N on the opposite wall, are zero), Neumann for a cell-centred one.
enum { SB_DIRICHLET_CELL = 1, SB_DIRICHLET_FACE = 2, SB_NEUMANN_CELL = 3 };

template <typename T>
struct SweepArgs {
  T *f[3];             // per field: right-hand side in
  T *o[3];             // PLAIN: solution out (may alias f)
  T *u[3];             // FINAL: u += x (per field)
  T *divn;             // PFINAL: D.u^{n+1} in
  T *divp;             // PFINAL: D.u^n in, D.u^{n+1} out
  double *p;           // PFINAL: p += x - chi mu (divn + divp)/2
  double alpha, inv_c; // factored-form coefficients (inv_c may carry a rhs scale)
  const double *alpha_layer, *invc_layer;  // 2-D batches: per-layer coefficients
  double half_chi_mu;  // PFINAL
  const double *gauge; // PFINAL: per-layer mean of psi removed before use (or null)
  double *gpart;       // PLAIN, 3-D: per-workgroup sums of the stored values (or null)
  int32_t bc[3];       // channel y sweeps: boundary kind per field (SB_*)
  Grid g;
  int32_t G;           // threads per line (x kernel: power of two <= 64)
  int32_t dim;
};

template <typename T, int MODE>
__device__ __forceinline__ void sweep_store(const SweepArgs<T> &a, int fld, int64_t idx,
                                            double x) {
  if (MODE == SW_PLAIN) {
    a.o[fld][idx] = (T)x;
  } else if (MODE == SW_FINAL) {
    a.u[fld][idx] = (T)((double)a.u[fld][idx] + x);
  } else {  // SW_PFINAL
    if (a.gauge) x -= a.gauge[a.dim == 2 ? idx / ((int64_t)a.g.n0 * a.g.n1) : 0];
    a.f[fld][idx] = (T)x;
    const T dn = a.divn[idx];
    const double dsum = (double)dn + (double)a.divp[idx];
    a.p[idx] = a.p[idx] + x - a.half_chi_mu * dsum;
    a.divp[idx] = dn;
  }
}

// Gauge partial sums fused into a plain psi sweep (FP32 work arrays): every
// workgroup adds the values it stores, as stored, in FP64, and writes the sum
// to part[1 + linear block index] (blockIdx.z, the field, is 0 for psi);
// block 0 also writes the block count to part[0], so k_layer_mean needs no
// count from the host.  In 2-D batches the host uses it only where every
// workgroup's lines lie in one layer, so a layer's sums are a contiguous
// run of count / layers.  Every thread of the block calls it, with
// v = 0 for threads that store nothing; the sums are taken in a fixed order
// (guarded lane reduction, then the waves in order).
__device__ __forceinline__ void block_sum_store(double v, double *part) {
  __shared__ double red[16];  // one per wave, at most 1024 threads
  const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
  const int nthr = blockDim.x * blockDim.y * blockDim.z;
  const int lane = tid & 63, wave = tid >> 6;
  const int wn = min(64, nthr - (wave << 6));  // lanes of this wave
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(v, off);
    if (lane + off < wn) v += o;
  }
  if (lane == 0) red[wave] = v;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int w = 0; w < (nthr + 63) / 64; w++) sum += red[w];
    const int64_t blk = blockIdx.x + (int64_t)gridDim.x * blockIdx.y;
    part[1 + blk] = sum;
    if (blk == 0) part[0] = (double)((int64_t)gridDim.x * gridDim.y);
  }
}

// 16-byte vector access to a full chunk of M consecutive values (host
// guarantees 16-byte alignment and M * sizeof(T) a multiple of 16).
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int n = 4;
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int n = 2;
};

template <typename T, int M>
__device__ __forceinline__ void vload(const T *p, double *r) {
  using V = typename Vec16<T>::type;
  constexpr int K = Vec16<T>::n;
#pragma unroll
  for (int v = 0; v < M / K; v++) {
    const V x = reinterpret_cast<const V *>(p)[v];
    const T *e = reinterpret_cast<const T *>(&x);
#pragma unroll
    for (int q = 0; q < K; q++) r[v * K + q] = (double)e[q];
  }
}

template <typename T, int M>
__device__ __forceinline__ void vstore(T *p, const double *r) {
  using V = typename Vec16<T>::type;
  constexpr int K = Vec16<T>::n;
#pragma unroll
  for (int v = 0; v < M / K; v++) {
    V x;
    T *e = reinterpret_cast<T *>(&x);
#pragma unroll
    for (int q = 0; q < K; q++) e[q] = (T)r[v * K + q];
    reinterpret_cast<V *>(p)[v] = x;
  }
}

// Contiguous (x) lines.  blockDim = 256; G lanes per line (power of two
// <= 64), each with a chunk of M consecutive elements; 256/G lines per block;
// blockIdx.y = field.  Chunks beyond the line end are empty (identity maps).
// VEC: every chunk is full and 16-byte aligned (N = G M), so chunks move
// with 16-byte vector loads and stores.
template <typename T, int M, int MODE, bool VEC>
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
  const int64_t lay = line / a.g.n1;
  const double al = a.alpha_layer ? a.alpha_layer[lay] : a.alpha;
  const double ic = a.invc_layer ? a.invc_layer[lay] : a.inv_c;

  double r[M];
  if (VEC) {
    vload<T, M>(a.f[fld] + base + s, r);
  } else {
#pragma unroll
    for (int q = 0; q < M; q++) r[q] = q < cnt ? (double)a.f[fld][base + s + q] : 0.0;
  }
  // forward recurrence over the chunk from zero
  double z = 0.0, A = 1.0;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (VEC || q < cnt) {
      z = al * z + r[q] * ic;
      r[q] = z;
      A *= al;
    }
  double B = z;
  double win;
  if (G == 64 || G == 32) {
    Aff ex, tot;
    if (G == 64) wave_prefix<64>(Aff{A, B}, ex, tot);
    else wave_prefix<32>(Aff{A, B}, ex, tot);
    win = ex.A * (tot.B / (1.0 - tot.A)) + ex.B;
  } else {
    // inclusive scan of the affine maps (earlier lanes act first)
    for (int off = 1; off < G; off <<= 1) {
      const double Ap = __shfl_up(A, off, G), Bp = __shfl_up(B, off, G);
      if (lane >= off) {
        B = A * Bp + B;
        A = A * Ap;
      }
    }
    const double At = __shfl(A, G - 1, G), Bt = __shfl(B, G - 1, G);
    const double wlast = Bt / (1.0 - At);
    double Ae = __shfl_up(A, 1, G), Be = __shfl_up(B, 1, G);
    if (lane == 0) {
      Ae = 1.0;
      Be = 0.0;
    }
    win = Ae * wlast + Be;
  }
  {
    // running product: one register instead of the M powers of al
    double cw = win;
#pragma unroll
    for (int q = 0; q < M; q++)
      if (VEC || q < cnt) {
        cw *= al;
        r[q] += cw;
      }
  }
  // backward recurrence over the chunk from zero
  double t = 0.0;
  A = 1.0;
#pragma unroll
  for (int q = M - 1; q >= 0; q--)
    if (VEC || q < cnt) {
      t = al * t + r[q];
      r[q] = t;
      A *= al;
    }
  B = t;
  double xin;
  if (G == 64 || G == 32) {
    Aff ex, tot;
    if (G == 64) wave_suffix<64>(Aff{A, B}, ex, tot);
    else wave_suffix<32>(Aff{A, B}, ex, tot);
    xin = ex.A * (tot.B / (1.0 - tot.A)) + ex.B;
  } else {
    // suffix scan (later lanes act first)
    for (int off = 1; off < G; off <<= 1) {
      const double An = __shfl_down(A, off, G), Bn = __shfl_down(B, off, G);
      if (lane + off < G) {
        B = A * Bn + B;
        A = A * An;
      }
    }
    const double A0 = __shfl(A, 0, G), B0 = __shfl(B, 0, G);
    const double x0 = B0 / (1.0 - A0);
    double An = __shfl_down(A, 1, G), Bn = __shfl_down(B, 1, G);
    if (lane == G - 1) {
      An = 1.0;
      Bn = 0.0;
    }
    xin = An * x0 + Bn;
  }
  {
    double cx = xin;
#pragma unroll
    for (int q = M - 1; q >= 0; q--)
      if (VEC || q < cnt) {
        cx *= al;
        r[q] += cx;
      }
  }
  if (MODE == SW_PLAIN && a.gpart) {
    double sum = 0.0;
    if (live)
#pragma unroll
      for (int q = 0; q < M; q++)
        if (VEC || q < cnt) sum += (double)(T)r[q];
    block_sum_store(sum, a.gpart);
  }
  if (!live) return;
  if (VEC) {
    const int64_t o = base + s;
    if (MODE == SW_PLAIN) {
      vstore<T, M>(a.o[fld] + o, r);
    } else if constexpr (MODE == SW_FINAL) {
      // epilogue operands are read only now (held from the start they would
      // cost M registers through both passes)
      double pre0[M];
      vload<T, M>(a.u[fld] + o, pre0);
#pragma unroll
      for (int q = 0; q < M; q++) pre0[q] += r[q];
      vstore<T, M>(a.u[fld] + o, pre0);
    } else if constexpr (MODE == SW_PFINAL) {
      double pre0[M], pre1[M], pre2[M];
      vload<T, M>(a.divn + o, pre0);
      vload<T, M>(a.divp + o, pre1);
      vload<double, M>(a.p + o, pre2);
      if (a.gauge) {
        const double gz = a.gauge[a.dim == 2 ? lay : 0];
#pragma unroll
        for (int q = 0; q < M; q++) r[q] -= gz;
      }
      vstore<T, M>(a.f[fld] + o, r);
#pragma unroll
      for (int q = 0; q < M; q++) pre2[q] = pre2[q] + r[q] - a.half_chi_mu * (pre0[q] + pre1[q]);
      vstore<double, M>(a.p + o, pre2);
      vstore<T, M>(a.divp + o, pre0);
    }
    return;
  }
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
  // 2-D batches sweep y only, so the remaining index is the layer
  const double al = a.alpha_layer ? a.alpha_layer[other] : a.alpha;
  const double ic = a.invc_layer ? a.invc_layer[other] : a.inv_c;
  const int slot = g * TX + tx;

  double r[M];
#pragma unroll
  for (int q = 0; q < M; q++) r[q] = q < cnt ? (double)a.f[fld][base + q * stride] : 0.0;
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
  if (MODE == SW_PLAIN && a.gpart) {
    double sum = 0.0;
    if (live)
#pragma unroll
      for (int q = 0; q < M; q++)
        if (q < cnt) sum += (double)(T)r[q];
    block_sum_store(sum, a.gpart);
  }
  if (!live) return;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (q < cnt) sweep_store<T, MODE>(a, fld, base + q * stride, r[q]);
}

// Strided lines through buffer resources.  blockDim = (TX, G): TX = 64 makes
// a wave one 64-wide row of x (256 or 512 contiguous bytes per access), TX =
// 32 halves the block for register-heavy FP64 recurrences; threadIdx.y is
// the chunk of M line elements.  Each array is addressed by a buffer resource
// based at the block's first column; a thread's lane and chunk start are one
// VGPR offset, and element q of its chunk adds q * stride, a scalar (q is a
// compile-time index), so no per-element addresses are held and no offset
// has to be made wave-uniform.  Reads past the end of an array return 0 and
// writes are dropped by the resource's range check.  Requires
// (N - 1) * stride * sizeof(double) + 64 * sizeof(double) < 2^31.
template <typename T>
struct Col {
  __amdgpu_buffer_rsrc_t r;
  int vo;  // byte offset of the thread's first element (lane + chunk start)
  int sb;  // byte stride between line elements
  __device__ __forceinline__ Col(const void *base, int64_t bytes, int lane, int64_t stride,
                                 int pos0) {
    const int64_t lim = bytes < 0x7fffffff ? bytes : 0x7fffffff;
    r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)lim, 0x00020000);
    sb = (int)(stride * (int64_t)sizeof(T));
    vo = lane * (int)sizeof(T) + pos0 * sb;
  }
  __device__ __forceinline__ T ld(int q) const {
    if constexpr (sizeof(T) == 4) {
      return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, q * sb, 0));
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, q * sb, 0);
      return __hiloint2double((int)v[1], (int)v[0]);
    }
  }
  __device__ __forceinline__ void st(int q, T x) const {
    if constexpr (sizeof(T) == 4) {
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, vo, q * sb, 0);
    } else {
      typedef unsigned int u2 __attribute__((ext_vector_type(2)));
      u2 v;
      v[0] = (unsigned)__double2loint(x);
      v[1] = (unsigned)__double2hiint(x);
      __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, q * sb, 0);
    }
  }
};

// The column solve of one chunk row: forward recurrence over the chunk from
// zero, the chunk maps of the rows above combined through LDS (sA, sB) and
// the periodic fixed point closed, then the same backward.  r holds the
// chunk's right-hand side in and its solution out.
template <typename R, int M, bool EVEN>
__device__ __forceinline__ void sb_solve(R (&r)[M], int cnt, R al, R ic, R *sA, R *sB, int g,
                                         int G, int TX, int tx) {
  const int slot = g * TX + tx;
  R z = 0, A = 1;
#pragma unroll
  for (int q = 0; q < M; q++)
    if (EVEN || q < cnt) {
      z = al * z + r[q] * ic;
      r[q] = z;
      A *= al;
    }
  sA[slot] = A;
  sB[slot] = z;
  __syncthreads();
  {
    R Ap = 1, Bp = 0;
    for (int h = 0; h < g; h++) {
      Bp = sA[h * TX + tx] * Bp + sB[h * TX + tx];
      Ap = sA[h * TX + tx] * Ap;
    }
    R At = Ap, Bt = Bp;
    for (int h = g; h < G; h++) {
      Bt = sA[h * TX + tx] * Bt + sB[h * TX + tx];
      At = sA[h * TX + tx] * At;
    }
    // the incoming value decays by al per element: a running product keeps
    // one register live instead of the M powers of al
    R cw = Ap * (Bt / (R(1) - At)) + Bp;
#pragma unroll
    for (int q = 0; q < M; q++)
      if (EVEN || q < cnt) {
        cw *= al;
        r[q] += cw;
      }
  }
  __syncthreads();
  R t = 0;
  A = 1;
#pragma unroll
  for (int q = M - 1; q >= 0; q--)
    if (EVEN || q < cnt) {
      t = al * t + r[q];
      r[q] = t;
      A *= al;
    }
  sA[slot] = A;
  sB[slot] = t;
  __syncthreads();
  {
    R As = 1, Bs = 0;
    for (int h = G - 1; h > g; h--) {
      Bs = sA[h * TX + tx] * Bs + sB[h * TX + tx];
      As = sA[h * TX + tx] * As;
    }
    R At = As, Bt = Bs;
    for (int h = g; h >= 0; h--) {
      Bt = sA[h * TX + tx] * Bt + sB[h * TX + tx];
      At = sA[h * TX + tx] * At;
    }
    R cx = As * (Bt / (R(1) - At)) + Bs;
#pragma unroll
    for (int q = M - 1; q >= 0; q--)
      if (EVEN || q < cnt) {
        cx *= al;
        r[q] += cx;
      }
  }
}

// R: recurrence type (double, or float for the benign momentum systems under
// the mixed policy).  EVEN: the line length is G * M, so every chunk is full
// and the per-element guards drop out.
template <typename T, typename R, int M, int MODE, int LB, int TX, bool EVEN>
__global__ void __launch_bounds__(LB) k_sweep_sb(SweepArgs<T> a, int axis) {
  __shared__ R sA[LB], sB[LB];
  const int tx = threadIdx.x, g = threadIdx.y, G = blockDim.y;
  const int64_t n0 = a.g.n0, n1 = a.g.n1, ncell = a.g.ncell;
  const int64_t x0 = (int64_t)blockIdx.x * TX;
  const int64_t other = blockIdx.y;
  const int fld = blockIdx.z;
  const int N = axis == 1 ? (int)n1 : (int)a.g.n2;
  const int64_t stride = axis == 1 ? n0 : n0 * n1;
  const int64_t tb = axis == 1 ? x0 + other * n0 * n1 : x0 + other * n0;  // first column
  const int64_t rem = ncell - tb;                                          // elements to the end
  const bool live = x0 + tx < n0;
  const int s = g * M;
  const int cnt = EVEN ? M : (s >= N ? 0 : (N - s < M ? N - s : M));
  // 2-D batches sweep y only, so the remaining index is the layer
  const R al = (R)(a.alpha_layer ? a.alpha_layer[other] : a.alpha);
  const R ic = (R)(a.invc_layer ? a.invc_layer[other] : a.inv_c);
  auto col = [&](const auto *base) {
    using E = std::remove_cv_t<std::remove_pointer_t<decltype(base)>>;
    return Col<E>(base + tb, rem * (int64_t)sizeof(E), tx, stride, s);
  };

  R r[M];
  {
    const auto cf = col(a.f[fld]);
#pragma unroll
    for (int q = 0; q < M; q++) r[q] = (EVEN || q < cnt) ? (R)cf.ld(q) : R(0);
  }
  sb_solve<R, M, EVEN>(r, cnt, al, ic, sA, sB, g, G, TX, tx);
  if (MODE == SW_PLAIN && a.gpart) {
    double sum = 0.0;
    if (live)
#pragma unroll
      for (int q = 0; q < M; q++)
        if (EVEN || q < cnt) sum += (double)(T)r[q];
    block_sum_store(sum, a.gpart);
  }
  if (!live) return;
  if (MODE == SW_PLAIN) {
    const auto co = col(a.o[fld]);
#pragma unroll
    for (int q = 0; q < M; q++)
      if (EVEN || q < cnt) co.st(q, (T)r[q]);
  } else if constexpr (MODE == SW_FINAL) {
    // epilogue operands are read only now: held from the start they would
    // cost M registers through both passes (fewer resident waves)
    const auto cu = col(a.u[fld]);
    T pu[M];
#pragma unroll
    for (int q = 0; q < M; q++) pu[q] = (EVEN || q < cnt) ? cu.ld(q) : T(0);
#pragma unroll
    for (int q = 0; q < M; q++)
      if (EVEN || q < cnt) cu.st(q, (T)((R)pu[q] + r[q]));
  } else if constexpr (MODE == SW_PFINAL) {
    if (a.gauge) {
      // 2-D batches sweep y only, so the remaining index is the layer
      const R gz = (R)a.gauge[a.dim == 2 ? other : 0];
#pragma unroll
      for (int q = 0; q < M; q++) r[q] -= gz;
    }
    const auto cf = col(a.f[fld]);
    const auto cdn = col(a.divn);
    const auto cdp = col(a.divp);
    const auto cp = col(a.p);
    T pdn[M], pdp[M];
    double pp[M];
#pragma unroll
    for (int q = 0; q < M; q++) {
      const bool in = EVEN || q < cnt;
      pdn[q] = in ? cdn.ld(q) : T(0);
      pdp[q] = in ? cdp.ld(q) : T(0);
      pp[q] = in ? cp.ld(q) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < M; q++)
      if (EVEN || q < cnt) {
        cf.st(q, (T)r[q]);
        cp.st(q, pp[q] + (double)r[q] - a.half_chi_mu * ((double)pdn[q] + (double)pdp[q]));
        cdp.st(q, pdn[q]);
      }
  }
}

// Channel y lines.  A bounded line of n1 elements is solved as the periodic
// line of 2 n1 that mirrors it (method of images): Dirichlet for a
// cell-centred unknown is the odd extension about the wall between cells,
// Neumann the even one, and Dirichlet for a face unknown on the wall the odd
// extension about that face (element 0 and element n1 then vanish).  The
// workgroup holds the virtual line: chunk rows 0 .. G/2-1 read the line,
// rows G/2 .. G-1 read it backwards with the sign of the extension, and only
// the first half stores.  32 columns per row; n1 is a multiple of M, so no
// chunk straddles the mirror.  blockIdx.y = z index (3-D) or layer (2-D).
template <typename T, typename R, int M, int MODE, int LB>
__global__ void __launch_bounds__(LB) k_sweep_wall(SweepArgs<T> a) {
  constexpr int TX = 32;
  __shared__ R sA[LB], sB[LB];
  const int tx = threadIdx.x, g = threadIdx.y, G = blockDim.y;
  const int64_t n0 = a.g.n0, n1 = a.g.n1, ncell = a.g.ncell;
  const int64_t x0 = (int64_t)blockIdx.x * TX;
  const int64_t other = blockIdx.y;
  const int fld = blockIdx.z;
  const int N = (int)n1;
  const int64_t tb = x0 + other * n0 * n1;  // first column of the block
  const int64_t rem = ncell - tb;
  const bool live = x0 + tx < n0;
  const int s = g * M;  // chunk start on the virtual line of 2N
  const bool mirror = s >= N;
  const int bc = a.bc[fld];
  const R al = (R)(a.alpha_layer ? a.alpha_layer[other] : a.alpha);
  const R ic = (R)(a.invc_layer ? a.invc_layer[other] : a.inv_c);
  // first real element of the chunk's span (backwards for mirrored chunks):
  // a mirrored cell chunk covers 2N-1-s .. 2N-s-M, a mirrored face chunk
  // 2N-s .. 2N-s-M+1 (its element at s = N is the far wall, zero)
  const int face = bc == SB_DIRICHLET_FACE;
  const int r0 = !mirror ? s : (face ? 2 * N - s - M + 1 : 2 * N - s - M);
  auto col = [&](const auto *base) {
    using E = std::remove_cv_t<std::remove_pointer_t<decltype(base)>>;
    return Col<E>(base + tb, rem * (int64_t)sizeof(E), tx, n0, r0);
  };
  R r[M];
  {
    const auto cf = col(a.f[fld]);
    if (!mirror) {
#pragma unroll
      for (int q = 0; q < M; q++) r[q] = (R)cf.ld(q);
    } else {
      const R sg = bc == SB_NEUMANN_CELL ? R(1) : R(-1);
#pragma unroll
      for (int q = 0; q < M; q++) {
        const R v = (R)cf.ld(M - 1 - q);
        r[q] = (face && q == 0 && s == N) ? R(0) : sg * v;
      }
    }
  }
  sb_solve<R, M, true>(r, M, al, ic, sA, sB, g, G, TX, tx);
  const bool wall0 = face && s == 0;  // element 0 is the wall face
  if (MODE == SW_PLAIN && a.gpart) {
    double sum = 0.0;
    if (live && !mirror)
#pragma unroll
      for (int q = 0; q < M; q++) sum += (q == 0 && wall0) ? 0.0 : (double)(T)r[q];
    block_sum_store(sum, a.gpart);
  }
  if (!live || mirror) return;
  if (MODE == SW_PLAIN) {
    const auto co = col(a.o[fld]);
#pragma unroll
    for (int q = 0; q < M; q++) co.st(q, (q == 0 && wall0) ? T(0) : (T)r[q]);
  } else if constexpr (MODE == SW_FINAL) {
    const auto cu = col(a.u[fld]);
    T pu[M];
#pragma unroll
    for (int q = 0; q < M; q++) pu[q] = cu.ld(q);
#pragma unroll
    for (int q = 0; q < M; q++)
      if (!(q == 0 && wall0)) cu.st(q, (T)((R)pu[q] + r[q]));
  } else if constexpr (MODE == SW_PFINAL) {
    if (a.gauge) {
      const R gz = (R)a.gauge[a.dim == 2 ? other : 0];
#pragma unroll
      for (int q = 0; q < M; q++) r[q] -= gz;
    }
    const auto cf = col(a.f[fld]);
    const auto cdn = col(a.divn);
    const auto cdp = col(a.divp);
    const auto cp = col(a.p);
    T pdn[M], pdp[M];
    double pp[M];
#pragma unroll
    for (int q = 0; q < M; q++) {
      pdn[q] = cdn.ld(q);
      pdp[q] = cdp.ld(q);
      pp[q] = cp.ld(q);
    }
#pragma unroll
    for (int q = 0; q < M; q++) {
      cf.st(q, (T)r[q]);
      cp.st(q, pp[q] + (double)r[q] - a.half_chi_mu * ((double)pdn[q] + (double)pdp[q]));
      cdp.st(q, pdn[q]);
    }
  }
}

// Gauge of psi.  On the periodic box the mean of psi is zero in exact
// arithmetic (the mean of D.u vanishes and every (1 - D_aa) maps a constant to
// itself), but with FP32 work arrays the rounding of D.u^{n+1} has a mean that
// the psi solve passes on multiplied by rho/dt, and p would accumulate it.
// These two kernels measure the mean of psi before the last sweep (which
// keeps the mean) per independent layer (one in 3-D), in FP64; the last
// sweep removes it.
template <typename T>
__global__ void __launch_bounds__(256) k_layer_partial(const T *f, int64_t per_layer,
                                                       double *partial) {
  __shared__ double red[256];
  const T *g = f + (int64_t)blockIdx.y * per_layer;
  double s = 0.0;
  // 16-byte loads where the layer is 16-byte aligned and a whole number of
  // vectors long (the FP32 3-D and power-of-two 2-D cases), else scalars
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::n;
  if (per_layer % VN == 0 && (reinterpret_cast<uintptr_t>(g) & 15) == 0) {
    const V *gv = reinterpret_cast<const V *>(g);
    const int64_t nv = per_layer / VN;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nv;
         i += (int64_t)gridDim.x * 256) {
      const V v = gv[i];
      if constexpr (VN == 4)
        s += ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
      else
        s += (double)v.x + (double)v.y;
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < per_layer;
         i += (int64_t)gridDim.x * 256)
      s += (double)g[i];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// One workgroup per layer: the mean of its nblk partial sums over per_layer
// cells.  Each thread keeps four loads in flight (four running sums, combined
// in a fixed order), so a few thousand partials take a couple of memory
// round trips rather than one per partial.
__global__ void __launch_bounds__(1024) k_layer_mean(const double *partial, int nblk,
                                                     int64_t per_layer, double *mean) {
  __shared__ double red[1024];
  if (nblk < 0) {  // partial sums written by a sweep (block_sum_store), layer by layer
    nblk = (int)partial[0] / (int)gridDim.x;
    partial += 1;
  }
  const double *pl = partial + (int64_t)blockIdx.x * nblk;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < nblk; i += 4 * 1024) {
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int j = i + u * 1024;
      if (j < nblk) s[u] += pl[j];
    }
  }
  red[threadIdx.x] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) mean[blockIdx.x] = red[0] / (double)per_layer;
}

// Grid-field watchdog: over every cell, bit 1 of *flags if a velocity
// component is non-finite, bit 2 if p is, and the largest |u| over all
// faces as the bit pattern of a non-negative double in *umax_bits (integer
// maximum = floating maximum for non-negative values).  Grid-stride; one
// atomic of each kind per wave.
template <typename V, int DIM>
__global__ void __launch_bounds__(256) k_field_check(const V *u0, const V *u1, const V *u2,
                                                     const double *p, int64_t ncell,
                                                     unsigned *flags,
                                                     unsigned long long *umax_bits) {
  double m = 0.0;
  unsigned f = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ncell;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double a = (double)u0[i], b = (double)u1[i], c = DIM == 3 ? (double)u2[i] : 0.0;
    if (!isfinite(a) || !isfinite(b) || !isfinite(c)) f |= 1u;
    if (!isfinite(p[i])) f |= 2u;
    m = fmax(m, fmax(fabs(a), fmax(fabs(b), fabs(c))));  // (fmax drops NaN)
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    m = fmax(m, __shfl_xor(m, off));
    f |= (unsigned)__shfl_xor((int)f, off);
  }
  if (__lane_id() == 0) {
    if (f) atomicOr(flags, f);
    atomicMax(umax_bits, (unsigned long long)__double_as_longlong(m));
  }
}

// Clear n 32-bit words (grid-stride): the fill kernel that clears counters
// and outputs in code a caller may capture into a graph, where memset nodes
// are avoided.
__global__ void __launch_bounds__(256) k_zero_words(uint32_t *p, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

}  // namespace ibgm
