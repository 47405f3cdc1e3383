// ibgm.hip -- host side of libibgm.so: the C ABI declared in include/ibgm.h.
//
// One translation unit: the device code lives in kernels.h.  The host only
// validates, precomputes the factored line-solve coefficients in extended
// precision, carves the caller's workspace and enqueues kernels on the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "errors.h"
#include "ibgm.h"
#include "kernels.h"

using namespace ibgm;

// ------------------------------------------------------------- errors --

static thread_local std::string g_err;

ib_status ibgm_err::fail(ib_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
using ibgm_err::fail;

#define HIP_TRY(expr)                                                     \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess)                                                 \
      return fail(IB_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

extern "C" const char *ib_last_error(void) { return g_err.c_str(); }

// --------------------------------------------------------- profiling --

enum KernelId {
  KP_INTERP_EVOLVE = 0, KP_FORCE, KP_SPREAD, KP_EXPLICIT, KP_DIVERGENCE,
  KP_MOM_X_PLAIN, KP_MOM_S_PLAIN, KP_MOM_X_FINAL, KP_MOM_S_FINAL,
  KP_PSI_X_FIRST, KP_PSI_S_FIRST, KP_PSI_X_PLAIN, KP_PSI_S_PLAIN,
  KP_PSI_X_PFINAL, KP_PSI_S_PFINAL, KP_LINE_X, KP_LINE_S, KP_INTERP, KP_SORT, KP_ADD, KP_GAUGE,
  KP_COUNT
};
static const char *kKernelNames[KP_COUNT] = {
    "interp_evolve", "force", "spread", "explicit", "divergence",
    "mom_x_plain", "mom_s_plain", "mom_x_final", "mom_s_final",
    "psi_x_first", "psi_s_first", "psi_x_plain", "psi_s_plain",
    "psi_x_pfinal", "psi_s_pfinal", "line_x", "line_s", "interp", "spread_sort", "add_increment",
    "psi_gauge"};

struct PendingEvent {
  int id;
  hipEvent_t a, b;
};

// ------------------------------------------------------------ context --

// Tile shapes of the sweep kernels picked by ib_tune (0 = default).
struct SweepTune {
  int x_m;        // elements per lane of x lines
  int s_tx, s_m;  // strided: row width and chunk length
};

struct ib_ctx {
  ib_grid_params prm;
  ib_buffers buf;
  hipStream_t stream;
  int64_t step;
  int dim;
  Grid g;
  int64_t np;
  bool f32;    // work arrays (N, psi, div, workspace) in FP32
  bool u64;    // velocity state in FP64 while the work arrays are FP32
  int resident3;  // workgroups of the 3-D explicit kernel resident on the device at once
  // Lagrangian work of the next step (Steps 1a-2b) overlapped with this
  // step's psi sweeps on a second stream: ev_u marks u^{n+1} final, ev_lag
  // the end of the overlapped work, lag_pending that it was enqueued
  hipStream_t stream2;
  hipEvent_t ev_u, ev_lag;
  bool lag_pending;
  size_t tsz;  // bytes per work-array value
  // workspace
  void *delta[3], *f[3], *divn;
  double *Xn1, *Xh, *F;
  int *flag;
  // spreading tiles
  TileGrid tg;
  int *t_count, *t_start, *t_flag, *t_bsum, *t_list, *t_nlist, *tile_of, *rank_of;
  int *point_of;  // deterministic spreading: the point in each sorted slot
  double *st_x;  // sorted point positions [dim][np]
  void *st_val;  // sorted spread values [dim][np] (grid dtype)
  // structure (library allocation)
  int32_t *ptr, *nbr;
  double *kap, *l0, *w;
  double *tk, *ty;  // tethers: stiffness [np] and target [dim][np] (null: none)
  int64_t nlinks;
  // factored coefficients
  double mom_alpha, mom_invc, psi_alpha, psi_invc;
  // 2-D batches (library allocation; null for single problems): layer of
  // each point, and per layer dt, momentum factors and the first psi sweep's
  // scaled 1/c
  int *p_layer;
  double *l_dt, *l_mom_alpha, *l_mom_invc, *l_psi_invc;
  // tile shapes chosen by ib_tune, per axis and recurrence type (0 = float)
  bool tuned;
  bool have_force;  // a step has spread its force into the workspace
  double *gauge, *gauge_part;  // psi means per layer and their partial sums
  SweepTune tune[3][2];
  // profiling
  bool prof;
  std::vector<PendingEvent> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[KP_COUNT];
  int64_t prof_n[KP_COUNT];
};

static hipEvent_t take_event(ib_ctx *c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Enqueue one kernel launch, bracketed by events while profiling.
template <class Fn>
static void launch(ib_ctx *c, int id, Fn &&fn) {
  hipEvent_t a = nullptr, b = nullptr;
  if (c && c->prof) {
    a = take_event(c);
    b = take_event(c);
    if (a) (void)hipEventRecord(a, c->stream);
  }
  fn();
  if (c && c->prof && a && b) {
    (void)hipEventRecord(b, c->stream);
    c->pending.push_back({id, a, b});
  }
}

static void drain_events(ib_ctx *c) {
  for (auto &p : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess &&
        hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->prof_ms[p.id] += ms;
      c->prof_n[p.id] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
}

// ------------------------------------------------- factored coefficients --

// A = d I + e (L + U) = c (I - alpha L)(I - alpha U) with |alpha| < 1:
// alpha + 1/alpha = -d/e.  With g = |d/e| - 2 > 0 (strict dominance), the
// smaller root is |alpha| = 2 / (2 + g + sqrt(g (g + 4))) (no cancellation
// for small or large g), sign(alpha) = sign(-d/e), c = -e/alpha.  Computed in
// long double from the given (d, e).
static ib_status factor(double d, double e, double *alpha, double *inv_c) {
  if (!std::isfinite(d) || !std::isfinite(e))
    return fail(IB_E_INVALID, "non-finite line-solve coefficients (%g, %g)", d, e);
  if (e == 0.0) {
    if (d == 0.0) return fail(IB_E_INVALID, "singular line-solve matrix (diag 0)");
    *alpha = 0.0;
    *inv_c = 1.0 / d;
    return IB_OK;
  }
  if (!(std::fabs(d) > 2.0 * std::fabs(e)))
    return fail(IB_E_INVALID,
                "line solve needs |diag| > 2|off| (got diag %g, off %g)", d, e);
  long double D = d, E = e;
  long double g = (fabsl(D) - 2.0L * fabsl(E)) / fabsl(E);
  long double aa = 2.0L / (2.0L + g + sqrtl(g * (g + 4.0L)));
  long double al = (-D / E) > 0 ? aa : -aa;
  long double c = -E / al;
  *alpha = (double)al;
  *inv_c = (double)(1.0L / c);
  return IB_OK;
}

// ----------------------------------------------------------- sweeps --

// Elements per lane of an x line: the smallest supported chunk that fits the
// line into 32 lanes, so a wave carries two lines (two loads in flight and
// two independent scans).
static int x_chunk(int64_t N) {
  static const int ms[] = {1, 2, 4, 6, 8, 12, 16, 32};
  for (int m : ms)
    if ((N + m - 1) / m <= 32) return m;
  return 32;
}
static int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

template <typename T, int M, int MODE, bool VEC>
static void go_x(SweepArgs<T> a, int nf, hipStream_t st) {
  int64_t nlines = (int64_t)a.g.n1 * a.g.n2;
  int lpb = 256 / a.G;
  dim3 grid((unsigned)((nlines + lpb - 1) / lpb), nf);
  hipLaunchKernelGGL((k_sweep_x<T, M, MODE, VEC>), grid, dim3(256), 0, st, a);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// Full, aligned chunks move as 16-byte vectors.
template <typename T, int MODE>
static bool x_vectorizable(const SweepArgs<T> &a, int nf, int M) {
  if ((int64_t)a.G * M != a.g.n0 || (M * (int)sizeof(T)) % 16 != 0 || (M * 8) % 16 != 0)
    return false;
  for (int i = 0; i < nf; i++) {
    if (!aligned16(a.f[i])) return false;
    if (MODE == SW_PLAIN && !aligned16(a.o[i])) return false;
    if (MODE == SW_FINAL && !aligned16(a.u[i])) return false;
  }
  if (MODE == SW_PFINAL && !(aligned16(a.divn) && aligned16(a.divp) && aligned16(a.p)))
    return false;
  return true;
}

template <typename T, int M, int MODE>
static void go_x_any(SweepArgs<T> a, int nf, hipStream_t st) {
  if constexpr ((M * sizeof(T)) % 16 == 0 && (M * 8) % 16 == 0) {
    if (x_vectorizable<T, MODE>(a, nf, M)) {
      go_x<T, M, MODE, true>(a, nf, st);
      return;
    }
  }
  go_x<T, M, MODE, false>(a, nf, st);
}

template <typename T, int MODE>
static void dispatch_x(SweepArgs<T> a, int nf, hipStream_t st, const SweepTune *tu = nullptr) {
  const int64_t N = a.g.n0;
  const int M = (tu && tu->x_m) ? tu->x_m : x_chunk(N);
  a.G = next_pow2((int)((N + M - 1) / M));
  switch (M) {
    case 1: go_x_any<T, 1, MODE>(a, nf, st); break;
    case 2: go_x_any<T, 2, MODE>(a, nf, st); break;
    case 4: go_x_any<T, 4, MODE>(a, nf, st); break;
    case 6: go_x_any<T, 6, MODE>(a, nf, st); break;
    case 8: go_x_any<T, 8, MODE>(a, nf, st); break;
    case 12: go_x_any<T, 12, MODE>(a, nf, st); break;
    case 16: go_x_any<T, 16, MODE>(a, nf, st); break;
    default: go_x_any<T, 32, MODE>(a, nf, st); break;
  }
}

// Strided lines (fallback for short lines or grids too large for 32-bit
// buffer offsets): chunks of 32 elements (8 for lines of at most 64), TX
// consecutive x per block row, ceil(N/M) rows; launch bound by block size.
template <typename T, int M, int MODE, int LB>
static void go_s(SweepArgs<T> a, int axis, int nf, int TX, hipStream_t st) {
  const int64_t N = axis == 1 ? a.g.n1 : a.g.n2;
  const int G = (int)((N + M - 1) / M);
  const int64_t other = axis == 1 ? a.g.n2 : a.g.n1;
  dim3 grid((unsigned)((a.g.n0 + TX - 1) / TX), (unsigned)other, nf);
  hipLaunchKernelGGL((k_sweep_s<T, M, MODE, LB>), grid, dim3(TX, G), 0, st, a, axis);
}

// Chunk length (16 or 32 line elements per thread) and row width (32 or 64
// columns) of the buffer-addressed strided sweep.  Defaults: chunk 16; rows
// of 64 for FP32 recurrences and of 32 for FP64 ones (whose larger register
// footprint otherwise leaves one block per compute unit).  IBGM_S_CHUNK and
// IBGM_S_TX override them for tuning runs.
static int env_choice(const char *name, int a, int b, int dflt) {
  const char *e = getenv(name);
  if (!e) return dflt;
  const int v = atoi(e);
  return v == a ? a : (v == b ? b : dflt);
}

template <typename T, typename R, int M, int MODE, int LB, int TX>
static void go_sb(SweepArgs<T> a, int axis, int nf, hipStream_t st) {
  const int64_t N = axis == 1 ? a.g.n1 : a.g.n2;
  const int G = (int)((N + M - 1) / M);
  const int64_t other = axis == 1 ? a.g.n2 : a.g.n1;
  dim3 grid((unsigned)((a.g.n0 + TX - 1) / TX), (unsigned)other, nf);
  if (N % M == 0)
    hipLaunchKernelGGL((k_sweep_sb<T, R, M, MODE, LB, TX, true>), grid, dim3(TX, G), 0, st, a, axis);
  else
    hipLaunchKernelGGL((k_sweep_sb<T, R, M, MODE, LB, TX, false>), grid, dim3(TX, G), 0, st, a, axis);
}

template <typename T, typename R, int M, int MODE, int TX>
static bool go_sb_fit(SweepArgs<T> a, int axis, int nf, hipStream_t st) {
  const int64_t N = axis == 1 ? a.g.n1 : a.g.n2;
  const int threads = TX * (int)((N + M - 1) / M);
  if (threads <= 256) go_sb<T, R, M, MODE, 256, TX>(a, axis, nf, st);
  else if (threads <= 512) go_sb<T, R, M, MODE, 512, TX>(a, axis, nf, st);
  else if (threads <= 1024) go_sb<T, R, M, MODE, 1024, TX>(a, axis, nf, st);
  else return false;
  return true;
}

template <typename T, int MODE, typename R>
static void dispatch_s(SweepArgs<T> a, int axis, int nf, hipStream_t st,
                       const SweepTune *tu = nullptr) {
  const int64_t N = axis == 1 ? a.g.n1 : a.g.n2;
  const int64_t stride = axis == 1 ? a.g.n0 : a.g.n0 * a.g.n1;
  const bool buf_ok = N >= 64 && N <= 1024 && a.g.n0 >= 64 &&
                      ((N - 1) * stride + 64) * (int64_t)sizeof(double) < 0x7fffffff;
  if (buf_ok) {
    const int M = (tu && tu->s_m) ? tu->s_m : env_choice("IBGM_S_CHUNK", 16, 32, 16);
    const int TX = (tu && tu->s_tx) ? tu->s_tx
                                    : env_choice("IBGM_S_TX", 32, 64, sizeof(R) == 8 ? 32 : 64);
    bool ok;
    if (M == 16)
      ok = TX == 32 ? go_sb_fit<T, R, 16, MODE, 32>(a, axis, nf, st)
                    : go_sb_fit<T, R, 16, MODE, 64>(a, axis, nf, st);
    else
      ok = TX == 32 ? go_sb_fit<T, R, 32, MODE, 32>(a, axis, nf, st)
                    : go_sb_fit<T, R, 32, MODE, 64>(a, axis, nf, st);
    if (ok) return;
    if (go_sb_fit<T, R, 32, MODE, 32>(a, axis, nf, st)) return;
  }
  const int TX = a.g.n0 >= 32 ? 32 : (a.g.n0 >= 16 ? 16 : 8);
  if (N <= 64) {
    const int G = (int)((N + 7) / 8);
    if (TX * G <= 256) go_s<T, 8, MODE, 256>(a, axis, nf, TX, st);
    else go_s<T, 8, MODE, 512>(a, axis, nf, TX, st);
    return;
  }
  const int threads = TX * (int)((N + 31) / 32);
  if (threads <= 256) go_s<T, 32, MODE, 256>(a, axis, nf, TX, st);
  else if (threads <= 512) go_s<T, 32, MODE, 512>(a, axis, nf, TX, st);
  else go_s<T, 32, MODE, 1024>(a, axis, nf, TX, st);
}

static const SweepTune *tune_of(const ib_ctx *c, int axis, bool r64) {
  return (c && c->tuned) ? &c->tune[axis][r64 ? 1 : 0] : nullptr;
}

// Lines per workgroup of the plain x sweep with FP64 recurrences (the psi
// sweeps), as dispatch_x chooses them.
static int x_lines_per_block(const ib_ctx *c, int64_t N) {
  const SweepTune *tu = tune_of(c, 0, true);
  const int M = (tu && tu->x_m) ? tu->x_m : x_chunk(N);
  return 256 / next_pow2((int)((N + M - 1) / M));
}

// Launch one sweep along `axis`; `id_x` / `id_s` name it for profiling (the
// strided id is id_x + 1).  R is the recurrence type of the strided kernel.
// Channel walls: the y systems are bounded (a.bc per field); they are
// solved as periodic systems on the mirrored line of length 2 n1 (chunks of
// 16, or 32 above n1 = 256; 32 columns per workgroup row).
template <typename T, typename R, int M, int MODE, int LB>
static void go_wall(SweepArgs<T> a, int nf, hipStream_t st) {
  const int G = 2 * a.g.n1 / M;
  dim3 grid((unsigned)((a.g.n0 + 31) / 32), (unsigned)a.g.n2, nf);
  hipLaunchKernelGGL((k_sweep_wall<T, R, M, MODE, LB>), grid, dim3(32, G), 0, st, a);
}

template <typename T, int MODE, typename R>
static void dispatch_wall(SweepArgs<T> a, int nf, hipStream_t st) {
  const int n1 = (int)a.g.n1;  // 32..512, checked at ib_init
  if (n1 <= 64) go_wall<T, R, 16, MODE, 256>(a, nf, st);
  else if (n1 <= 128) go_wall<T, R, 16, MODE, 512>(a, nf, st);
  else if (n1 <= 256) go_wall<T, R, 16, MODE, 1024>(a, nf, st);
  else go_wall<T, R, 32, MODE, 1024>(a, nf, st);
}

template <typename T, int MODE, typename R = double>
static void sweep(ib_ctx *c, int id_x, SweepArgs<T> a, int axis, int nf, hipStream_t st) {
  // the tuner times plain sweeps; the sweeps with epilogue operands (FINAL,
  // PFINAL) hold more registers per element and keep the library's shapes
  const SweepTune *tu = MODE == SW_PLAIN ? tune_of(c, axis, sizeof(R) == 8) : nullptr;
  if (axis == 1 && c && (c->prm.flags & IB_FLAG_WALLS_Y)) {  // (ib_line_solve: no context)
    launch(c, id_x + 1, [&] { dispatch_wall<T, MODE, R>(a, nf, st); });
    return;
  }
  if (axis == 0)
    launch(c, id_x, [&] { dispatch_x<T, MODE>(a, nf, st, tu); });
  else
    launch(c, id_x + 1, [&] { dispatch_s<T, MODE, R>(a, axis, nf, st, tu); });
}

// ------------------------------------------------------------ validation --

static bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

static ib_status check_params(const ib_grid_params *p) {
  if (!p) return fail(IB_E_INVALID, "null parameters");
  if (p->dim != 2 && p->dim != 3) return fail(IB_E_INVALID, "dim must be 2 or 3 (got %d)", p->dim);
  for (int a = 0; a < p->dim; a++)
    if (p->n[a] < 4 || p->n[a] > 1024)
      return fail(IB_E_INVALID, "n[%d] = %d outside [4, 1024]", a, p->n[a]);
  if (p->dim == 2 && (p->n[2] < 1 || p->n[2] > 65535))
    return fail(IB_E_INVALID, "2-D layer count n[2] = %d outside [1, 65535]", p->n[2]);
  if (p->dim == 2 && p->layer_dt)
    for (int l = 0; l < p->n[2]; l++)
      if (!finite_pos(p->layer_dt[l]))
        return fail(IB_E_INVALID, "layer_dt[%d] must be finite and > 0", l);
  if (!finite_pos(p->h)) return fail(IB_E_INVALID, "h must be finite and > 0");
  if (!finite_pos(p->rho)) return fail(IB_E_INVALID, "rho must be finite and > 0");
  if (!finite_pos(p->dt)) return fail(IB_E_INVALID, "dt must be finite and > 0");
  if (!(std::isfinite(p->mu) && p->mu >= 0)) return fail(IB_E_INVALID, "mu must be finite and >= 0");
  if (!(std::isfinite(p->chi) && p->chi >= 0 && p->chi <= 1))
    return fail(IB_E_INVALID, "chi must lie in [0, 1]");
  if (p->precision != IB_PREC_FP64 && p->precision != IB_PREC_MIXED &&
      p->precision != IB_PREC_MIXED_STATE64)
    return fail(IB_E_INVALID, "unknown precision %d", p->precision);
  if (p->step0 < 0) return fail(IB_E_INVALID, "step0 must be >= 0");
  for (int a = 0; a < 3; a++)
    if (!std::isfinite(p->body_force[a])) return fail(IB_E_INVALID, "body_force must be finite");
  for (int a = 0; a < 3; a++) {
    if (!std::isfinite(p->wall_velocity[a]))
      return fail(IB_E_INVALID, "wall_velocity must be finite");
    if (p->wall_velocity[a] != 0.0 && (!(p->flags & IB_FLAG_WALLS_Y) || a == 1 || a >= p->dim))
      return fail(IB_E_INVALID,
                  "wall_velocity needs IB_FLAG_WALLS_Y and is tangential (x, and z in 3-D)");
  }
  if (p->flags & ~(IB_FLAG_NO_ADVECTION | IB_FLAG_WALLS_Y | IB_FLAG_DETERMINISTIC_SPREAD))
    return fail(IB_E_INVALID, "unknown flags 0x%x", p->flags);
  if (p->flags & IB_FLAG_WALLS_Y) {
    const int n1 = p->n[1];
    if (n1 < 32 || n1 > 512 || n1 % 16 != 0 || (n1 > 256 && n1 % 32 != 0))
      return fail(IB_E_INVALID,
                  "walls need 32 <= n[1] <= 512, a multiple of 16 (of 32 above 256); got %d", n1);
  }
  return IB_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static TileGrid tile_grid(const ib_grid_params *p) {
  TileGrid tg{};
  for (int a = 0; a < 3; a++) tg.nt[a] = a < p->dim ? (p->n[a] + TS - 1) / TS : p->n[a];
  tg.ntiles = (int64_t)tg.nt[0] * tg.nt[1] * tg.nt[2];
  return tg;
}

// Workspace: delta[3], f[3], div_new (grid dtype); X^{n+1}, X^{n+1/2}, F
// (FP64 [dim][np]); the points in sorted order (positions, spread values);
// the spreading tile tables (counts, flags, touched list, starts, block
// sums), the point sort (tile,
// rank, and the point of each slot in the deterministic order); the
// touched-list length; one status word.
// psi gauge (mixed policies): per layer, gauge_blocks() partial sums and the mean
static int64_t gauge_layers(const ib_grid_params *p) { return p->dim == 2 ? p->n[2] : 1; }
static int64_t gauge_blocks(int64_t per_layer) {  // ~4096 values per block, 1..4096 blocks
  const int64_t nb = (per_layer + 4095) / 4096;
  return nb < 1 ? 1 : (nb > 4096 ? 4096 : nb);
}
// The psi sweep before the last writes one partial sum per workgroup, after
// a count (block_sum_store): at most n1 n2 workgroups for x lines (four or
// more lines each), ceil(n0/8) max(n1, n2) for strided ones (n2 = layers in
// 2-D).
static int64_t gauge_sweep_parts(const ib_grid_params *p) {
  const int64_t n0 = p->n[0], n1 = p->n[1], n2 = p->n[2];
  return 1 + std::max<int64_t>(n1 * n2, ((n0 + 7) / 8) * std::max<int64_t>(n1, n2));
}
static size_t gauge_bytes(const ib_grid_params *p) {
  const int64_t L = gauge_layers(p);
  const int64_t per = (int64_t)p->n[0] * p->n[1] * (p->dim == 2 ? 1 : p->n[2]);
  const int64_t parts = std::max(L * gauge_blocks(per), gauge_sweep_parts(p));
  return align256(sizeof(double) * (size_t)(L + parts));
}

static size_t workspace_bytes(const ib_grid_params *p, int64_t np) {
  const size_t nc = (size_t)p->n[0] * p->n[1] * p->n[2];
  const size_t t = p->precision == IB_PREC_FP64 ? 8 : 4;
  const size_t npp = (size_t)(np > 0 ? np : 1);
  const size_t lag = sizeof(double) * (size_t)p->dim * npp;
  const TileGrid tg = tile_grid(p);
  const size_t nb = (size_t)((tg.ntiles + SCAN_TILE - 1) / SCAN_TILE);
  return 7 * align256(nc * t) + 3 * align256(lag) + align256(sizeof(double) * 3 * npp) +
         align256(t * 3 * npp) + 3 * align256(sizeof(int) * tg.ntiles) +
         align256(sizeof(int) * (tg.ntiles + 1)) + align256(sizeof(int) * nb) +
         3 * align256(sizeof(int) * npp) + 256 + 256 + gauge_bytes(p);
}

extern "C" ib_status ib_workspace_size(const ib_grid_params *prm, int64_t n_points,
                                       size_t *bytes) {
  ib_status st = check_params(prm);
  if (st != IB_OK) return st;
  if (n_points < 0) return fail(IB_E_INVALID, "n_points < 0");
  if (n_points > IB_MAX_POINTS) return fail(IB_E_UNSUPPORTED, "n_points above IB_MAX_POINTS");
  if (!bytes) return fail(IB_E_INVALID, "null output");
  *bytes = workspace_bytes(prm, n_points);
  return IB_OK;
}

// ---------------------------------------------------------- launches --

template <typename T, int DIM>
static void launch_interp(ib_ctx *c, int id, const double *X, int64_t np,
                          void *const u[3], double *U, bool evolve, bool first) {
  InterpArgs<T, DIM> a{};
  for (int i = 0; i < 3; i++) a.u[i] = (const T *)(i < DIM ? u[i] : nullptr);
  a.X = X;
  a.U = U;
  a.Xn1 = c->Xn1;
  a.Xh = c->Xh;
  a.flag = c->flag;
  a.layer = c->p_layer;
  a.dt_layer = c->l_dt;
  a.np = np;
  a.g = c->g;
  a.inv_h = 1.0 / c->prm.h;
  a.dt = c->prm.dt;
  a.evolve = evolve;
  a.first = first;
  // four lanes per (point, component), one stencil column each (k_interp)
  dim3 grid((unsigned)((4 * np + 255) / 256), DIM);
  launch(c, id, [&] {
    hipLaunchKernelGGL((k_interp<T, DIM>), grid, dim3(256), 0, c->stream, a);
  });
}

template <int DIM>
static void launch_force(ib_ctx *c, const double *Xh, double *F, bool commit,
                         bool bin = false) {
  ForceArgs<DIM> a{};
  a.ptr = c->ptr;
  a.nbr = c->nbr;
  a.kap = c->kap;
  a.l0 = c->l0;
  a.Xh = Xh;
  a.F = F;
  a.Xn1 = commit ? c->Xn1 : nullptr;
  a.X = c->buf.X;
  a.np = c->np;
  a.tk = c->tk;
  a.ty = c->ty;
  for (int i = 0; i < DIM; i++) a.box[i] = c->prm.n[i] * c->prm.h;
  launch(c, KP_FORCE, [&] {
    if (bin)  // also the spreading tiles and ranks of the points at Xh
      hipLaunchKernelGGL((k_force_bin<DIM>), dim3((unsigned)((c->np + 255) / 256)), dim3(256), 0,
                         c->stream, a, c->p_layer, c->g, c->tg, 1.0 / c->prm.h, c->t_count,
                         c->tile_of, c->rank_of);
    else
      hipLaunchKernelGGL((k_force<DIM>), dim3((unsigned)((c->np + 255) / 256)), dim3(256), 0,
                         c->stream, a);
  });
}

// Step 2b: sort the points into spreading tiles (gathering them in sorted
// order), list the tiles their stencils reach, then gather per tile.
// ADD = false: f = spread force on listed tiles and flags for the explicit
// step (the step's own buffers); ADD = true: f += spread force (the public
// entry point).
template <typename T, int DIM, bool ADD>
static void launch_spread(ib_ctx *c, const double *X, const double *F, const double *w,
                          int64_t np, void *const f[3], bool binned = false) {
  const double inv_h = 1.0 / c->prm.h;
  const unsigned pb = (unsigned)((np + 255) / 256);
  const unsigned nb = (unsigned)((c->tg.ntiles + SCAN_TILE - 1) / SCAN_TILE);
  if (!binned)  // (binned: k_force_bin has placed the points in their tiles)
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL((k_bin<DIM>), dim3(pb), dim3(256), 0, c->stream, X, c->p_layer, np,
                         c->g, c->tg, inv_h, c->t_count, c->tile_of, c->rank_of);
    });
  if (c->tg.ntiles <= SCAN_ONE_MAX) {
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(SCAN_ONE_THREADS), 0, c->stream, c->t_count,
                         c->t_start, c->tg.ntiles, c->t_nlist);
    });
  } else {
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(256), 0, c->stream, c->t_count, c->t_bsum,
                         c->tg.ntiles);
    });
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL(k_scan_bsums, dim3(1), dim3(256), 0, c->stream, c->t_bsum, (int)nb,
                         c->t_nlist);
    });
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL(k_scan_write, dim3(nb), dim3(256), 0, c->stream, c->t_count,
                         c->t_start, c->t_bsum, c->tg.ntiles);
    });
  }
  Sorted<T> stn{c->st_x, (T *)c->st_val};
  const double inv_hd = 1.0 / std::pow(c->prm.h, DIM);
  const unsigned tb = (unsigned)((c->tg.ntiles + 255) / 256);
  const bool det = (c->prm.flags & IB_FLAG_DETERMINISTIC_SPREAD) != 0;
  if (det) {  // each tile's points in point-index order
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL(k_place, dim3(pb), dim3(256), 0, c->stream, c->tile_of, c->rank_of,
                         c->t_start, c->point_of, np);
    });
    launch(c, KP_SORT, [&] {
      hipLaunchKernelGGL(k_order_tiles, dim3(tb), dim3(256), 0, c->stream, c->t_start,
                         c->point_of, c->tg.ntiles);
    });
  }
  // placing the points and listing the touched tiles, one launch
  launch(c, KP_SORT, [&] {
    hipLaunchKernelGGL((k_scatter_touch<T, DIM>), dim3(pb + tb), dim3(256), 0, c->stream,
                       c->tile_of, c->rank_of, c->t_start, det ? c->point_of : nullptr, X, F, w,
                       stn, c->g, inv_hd, np, (int)pb, ADD ? nullptr : c->t_flag,
                       c->t_list, c->t_nlist, c->tg);
  });
  SpreadArgs<T, DIM> a{};
  a.st = stn;
  a.inv_h = inv_h;
  for (int i = 0; i < 3; i++) a.f[i] = (T *)(i < DIM ? f[i] : nullptr);
  a.start = c->t_start;
  a.list = c->t_list;
  a.nlist = c->t_nlist;
  a.np = np;
  a.g = c->g;
  a.tg = c->tg;
  const unsigned grid = (unsigned)std::min<int64_t>(c->tg.ntiles, 4096);
  // Threads per touched tile: 1024 for a dense structure (over four points
  // per tile of the grid) on a grid of at most 8192 tiles (up to 160^3 in
  // 3-D), where the few touched tiles would leave the GPU half idle with
  // 256-thread workgroups; 256 otherwise -- on larger grids a dense
  // structure touches enough tiles, and smaller workgroups contend less for
  // each tile's LDS sums.  Measured: the 933,888-point cylinder at 256^3
  // (28 points per tile) 1.354 -> 1.247 ms per step with 256; at 128^3
  // 0.343 (1024) vs 0.360 ms (256); the closure's 128^3 coarse step 0.269
  // (1024) vs 0.344 ms (256).
  const bool dense = np > 4 * c->tg.ntiles && c->tg.ntiles <= 8192;
  launch(c, KP_SPREAD, [&] {
    if (det)
      hipLaunchKernelGGL((k_spread_det<T, DIM, ADD>), dim3(grid), dim3(256), 0, c->stream, a);
    else if (dense)
      hipLaunchKernelGGL((k_spread_tiles<T, DIM, ADD, 1024>), dim3(grid), dim3(1024), 0, c->stream, a);
    else
      hipLaunchKernelGGL((k_spread_tiles<T, DIM, ADD, 256>), dim3(grid), dim3(256), 0, c->stream, a);
  });
}

// Grid of the per-cell kernels: blocks of 64 x 4 cells over (x, y), one
// z-plane (or 2-D layer) per blockIdx.z.
static dim3 cell_grid(const Grid &g) {
  return dim3((unsigned)((g.n0 + 63) / 64), (unsigned)((g.n1 + 3) / 4), (unsigned)g.n2);
}

template <typename T, int DIM, typename V = T>
static ExplicitArgs<T, DIM, V> explicit_args(ib_ctx *c, bool first) {
  ExplicitArgs<T, DIM, V> a{};
  for (int i = 0; i < 3; i++) {
    a.u[i] = (const V *)(i < DIM ? c->buf.u[i] : nullptr);
    a.nl[i] = (T *)(i < DIM ? c->buf.nl_prev[i] : nullptr);
    a.f[i] = (const T *)(i < DIM ? c->f[i] : nullptr);
    a.delta[i] = (T *)(i < DIM ? c->delta[i] : nullptr);
  }
  a.p = c->buf.p;
  a.psi = (const T *)c->buf.psi;
  a.flag = c->t_flag;
  a.dt_layer = c->l_dt;
  a.g = c->g;
  a.tg = c->tg;
  a.inv_h = 1.0 / c->prm.h;
  a.inv_h2 = 1.0 / (c->prm.h * c->prm.h);
  a.dt = c->prm.dt;
  a.mu = c->prm.mu;
  a.inv_rho = 1.0 / c->prm.rho;
  a.first = first;
  a.advect = !(c->prm.flags & IB_FLAG_NO_ADVECTION);
  a.walls = (c->prm.flags & IB_FLAG_WALLS_Y) ? 1 : 0;
  for (int i = 0; i < 3; i++) a.g_body[i] = i < DIM ? c->prm.body_force[i] : 0.0;
  for (int i = 0; i < 3; i++) a.wall_u[i] = i < DIM ? c->prm.wall_velocity[i] : 0.0;
  return a;
}

template <typename T, int DIM, typename V = T>
static void launch_explicit(ib_ctx *c, bool first) {
  ExplicitArgs<T, DIM, V> a = explicit_args<T, DIM, V>(c, first);
  if constexpr (DIM == 3) {
    if (c->g.n0 % EX == 0 && c->g.n1 % EY == 0 && c->g.ncell < INT32_MAX) {
      // one round of resident workgroups (c->resident3, from ib_init) split
      // over the (x, y) column tiles
      const int resident = std::max(1, c->resident3);
      const int64_t cols = (c->g.n0 / EX) * (c->g.n1 / EY);
      const int64_t zb = std::max<int64_t>(1, std::min<int64_t>(c->g.n2, resident / cols));
      a.ez = (int)((c->g.n2 + zb - 1) / zb);
      const int64_t nblk = cols * ((c->g.n2 + a.ez - 1) / a.ez);
      launch(c, KP_EXPLICIT, [&] {
        hipLaunchKernelGGL((k_explicit3<T, V>), dim3((unsigned)nblk), dim3(EX * EY), 0, c->stream, a);
      });
      return;
    }
  }
  launch(c, KP_EXPLICIT, [&] {
    hipLaunchKernelGGL((k_explicit<T, DIM, V>), cell_grid(c->g), dim3(64, 4), 0, c->stream, a);
  });
}

// D.u of the velocity state (type V) into `out` (work type T).
template <typename T, int DIM, typename V = T>
static void launch_divergence(ib_ctx *c, void *out) {
  const bool vec = c->g.n0 % 4 == 0 && aligned16(out) && aligned16(c->buf.u[0]) &&
                   aligned16(c->buf.u[1]) && (DIM == 2 || aligned16(c->buf.u[2]));
  if (vec) {
    const dim3 grid((unsigned)((c->g.n0 / 4 + 63) / 64), (unsigned)((c->g.n1 + 3) / 4),
                    (unsigned)c->g.n2);
    launch(c, KP_DIVERGENCE, [&] {
      hipLaunchKernelGGL((k_divergence4<V, DIM, T>), grid, dim3(64, 4), 0, c->stream,
                         (const V *)c->buf.u[0], (const V *)c->buf.u[1],
                         (const V *)(DIM == 3 ? c->buf.u[2] : nullptr), (T *)out, c->g,
                         1.0 / c->prm.h);
    });
    return;
  }
  launch(c, KP_DIVERGENCE, [&] {
    hipLaunchKernelGGL((k_divergence<V, DIM, T>), cell_grid(c->g),
                       dim3(64, 4), 0, c->stream, (const V *)c->buf.u[0],
                       (const V *)c->buf.u[1], (const V *)(DIM == 3 ? c->buf.u[2] : nullptr),
                       (T *)out, c->g, 1.0 / c->prm.h);
  });
}

// div_prev = D.u^0 at a fresh start.
static void seed_divergence(ib_ctx *c) {
  void *o = c->buf.div_prev;
  if (c->u64) {
    if (c->dim == 2) launch_divergence<float, 2, double>(c, o);
    else launch_divergence<float, 3, double>(c, o);
  } else if (c->f32) {
    if (c->dim == 2) launch_divergence<float, 2>(c, o);
    else launch_divergence<float, 3>(c, o);
  } else {
    if (c->dim == 2) launch_divergence<double, 2>(c, o);
    else launch_divergence<double, 3>(c, o);
  }
}

// Steps 1a-2b of the step at hand: interpolation and position update, link
// force (committing X^{n+1}), spreading.  T: work arrays; V: velocity state.
template <typename T, int DIM, typename V = T>
static void enqueue_lagrangian(ib_ctx *c, bool first) {
  // Steps 1a-1c
  launch_interp<V, DIM>(c, KP_INTERP_EVOLVE, c->buf.X, c->np, c->buf.u, c->buf.U_prev,
                        true, first);
  // Step 2a (+ commit X^{n+1}, + the points' spreading tiles) and Step 2b
  launch_force<DIM>(c, c->Xh, c->F, true, true);
  launch_spread<T, DIM, false>(c, c->Xh, c->F, c->w, c->np, c->f, true);
}

// One full IB-GM step (Steps 1a-3f) at step index n.  T: work arrays; V:
// velocity state (V = double with T = float is the FP64-state policy: the
// last momentum sweep then leaves its increment in the work array and
// u += d runs in FP64).  With `overlap` (another step follows in the same
// enqueue), the next step's Steps 1a-2b -- which need only u^{n+1} and
// X^{n+1}, and touch none of the fields of Steps 3e-3f -- are enqueued on
// the second stream as soon as u^{n+1} is final and run beside this step's
// divergence and psi sweeps; the next step joins them before its explicit
// step.
template <typename T, int DIM, typename V>
static void enqueue_step(ib_ctx *c, bool overlap) {
  constexpr bool kState64 = !std::is_same<T, V>::value;
  const int64_t n = c->step;
  const bool first = n == 0;
  if (c->lag_pending) {
    (void)hipStreamWaitEvent(c->stream, c->ev_lag, 0);
    c->lag_pending = false;
  } else {
    enqueue_lagrangian<T, DIM, V>(c, first);
  }
  // split order of this step
  int order[3];
  const int shift = c->prm.rotate_split ? (int)(n % DIM) : 0;
  for (int s = 0; s < DIM; s++) order[s] = (s + shift) % DIM;
  // Steps 3a-3b
  launch_explicit<T, DIM, V>(c, first);
  // Steps 3c-3d (+z): delta form (1 - nu D_aa) d_a = d_{a-1}, u += d_last;
  // the momentum systems are well conditioned (|alpha| well below 1), so
  // their strided recurrences run in the storage precision
  SweepArgs<T> m{};
  m.g = c->g;
  m.dim = DIM;
  m.alpha = c->mom_alpha;
  m.inv_c = c->mom_invc;
  m.alpha_layer = c->l_mom_alpha;
  m.invc_layer = c->l_mom_invc;
  for (int i = 0; i < 3; i++) {
    m.f[i] = m.o[i] = (T *)(i < DIM ? c->delta[i] : nullptr);
    m.u[i] = kState64 ? nullptr : (T *)(i < DIM ? c->buf.u[i] : nullptr);
    m.bc[i] = i == 1 ? SB_DIRICHLET_FACE : SB_DIRICHLET_CELL;  // used by wall sweeps only
  }
  for (int s = 0; s < DIM; s++) {
    if (s < DIM - 1 || kState64) sweep<T, SW_PLAIN, T>(c, KP_MOM_X_PLAIN, m, order[s], DIM, c->stream);
    else sweep<T, SW_FINAL, T>(c, KP_MOM_X_FINAL, m, order[s], DIM, c->stream);
  }
  if constexpr (kState64) {
    launch(c, KP_ADD, [&] {
      hipLaunchKernelGGL((k_add_increment<T, DIM>), dim3((unsigned)((c->g.ncell + 255) / 256)),
                         dim3(256), 0, c->stream, (double *)c->buf.u[0], (double *)c->buf.u[1],
                         (double *)(DIM == 3 ? c->buf.u[2] : c->buf.u[0]), (const T *)c->delta[0],
                         (const T *)c->delta[1], (const T *)(DIM == 3 ? c->delta[2] : c->delta[0]),
                         c->g.ncell);
    });
  }
  if (overlap) {
    // fork: the next step's Lagrangian work on the second stream
    hipStream_t main = c->stream;
    (void)hipEventRecord(c->ev_u, main);
    (void)hipStreamWaitEvent(c->stream2, c->ev_u, 0);
    c->stream = c->stream2;
    enqueue_lagrangian<T, DIM, V>(c, false);
    c->stream = main;
    (void)hipEventRecord(c->ev_lag, c->stream2);
    c->lag_pending = true;
  }
  // Steps 3e-3f: D.u^{n+1} into div_new, then the psi sweeps: the first
  // solves for -(rho/dt) div_new (the scale rides on 1/c) into psi, the last
  // also updates p and hands div_new to div_prev
  launch_divergence<T, DIM, V>(c, c->divn);
  SweepArgs<T> q{};
  q.g = c->g;
  q.dim = DIM;
  q.alpha = c->psi_alpha;
  q.inv_c = c->psi_invc * (-c->prm.rho / c->prm.dt);
  q.invc_layer = c->l_psi_invc;  // per-layer -(rho/dt)/c in 2-D batches
  q.f[0] = (T *)c->divn;
  q.o[0] = (T *)c->buf.psi;
  q.bc[0] = SB_NEUMANN_CELL;  // used by wall sweeps only
  // FP32 work arrays: the mean of psi (zero in exact arithmetic) is measured
  // before the last sweep, which removes it.  The sweep before the last (the
  // middle one in 3-D, the first in 2-D) adds up the values it stores per
  // workgroup, so no pass of its own reads psi again; in 2-D batches every
  // workgroup's lines must lie in one layer (strided sweeps: always; x lines:
  // when the lines per workgroup divide n1), else a separate pass sums psi.
  bool fused_gauge = c->f32;
  if (fused_gauge && DIM == 2 && order[0] == 0)
    fused_gauge = c->g.n1 % x_lines_per_block(c, c->g.n0) == 0;
  q.gpart = (fused_gauge && DIM == 2) ? c->gauge_part : nullptr;
  sweep<T, SW_PLAIN>(c, KP_PSI_X_FIRST, q, order[0], 1, c->stream);
  q.gpart = nullptr;
  q.inv_c = c->psi_invc;
  q.invc_layer = nullptr;
  q.f[0] = q.o[0] = (T *)c->buf.psi;
  q.divn = (T *)c->divn;
  q.divp = (T *)c->buf.div_prev;
  q.p = c->buf.p;
  q.half_chi_mu = 0.5 * c->prm.chi * c->prm.mu;
  for (int s = 1; s < DIM - 1; s++) {
    q.gpart = fused_gauge ? c->gauge_part : nullptr;
    sweep<T, SW_PLAIN>(c, KP_PSI_X_PLAIN, q, order[s], 1, c->stream);
    q.gpart = nullptr;
  }
  if (c->f32) {
    const int64_t layers = DIM == 2 ? c->g.n2 : 1;
    const int64_t per = c->g.ncell / layers;
    const int64_t nb = gauge_blocks(per);
    launch(c, KP_GAUGE, [&] {
      if (!fused_gauge)
        hipLaunchKernelGGL((k_layer_partial<T>), dim3((unsigned)nb, (unsigned)layers), dim3(256),
                           0, c->stream, (const T *)c->buf.psi, per, c->gauge_part);
      hipLaunchKernelGGL(k_layer_mean, dim3((unsigned)layers), dim3(1024), 0, c->stream,
                         (const double *)c->gauge_part, fused_gauge ? -1 : (int)nb, per, c->gauge);
    });
    q.gauge = c->gauge;
  }
  sweep<T, SW_PFINAL>(c, KP_PSI_X_PFINAL, q, order[DIM - 1], 1, c->stream);
  c->step = n + 1;
  c->have_force = true;
}

static void enqueue_any(ib_ctx *c, bool overlap);

// ---------------------------------------------------------------- API --

extern "C" ib_status ib_init(ib_ctx **out, const ib_grid_params *prm, const ib_buffers *buf,
                             const ib_structure *st, void *hip_stream) {
  if (!out) return fail(IB_E_INVALID, "null context output");
  *out = nullptr;
  ib_status s = check_params(prm);
  if (s != IB_OK) return s;
  if (!buf || !st) return fail(IB_E_INVALID, "null buffers / structure");
  const int d = prm->dim;
  for (int c = 0; c < d; c++)
    if (!buf->u[c] || !buf->nl_prev[c]) return fail(IB_E_INVALID, "null velocity buffer %d", c);
  if (!buf->psi || !buf->div_prev || !buf->p) return fail(IB_E_INVALID, "null p / psi / div_prev");
  const int64_t np = buf->n_points;
  if (np < 1) return fail(IB_E_INVALID, "n_points must be >= 1");
  if (np > IB_MAX_POINTS)
    return fail(IB_E_UNSUPPORTED, "n_points = %lld above %lld (32-bit sort ranks)", (long long)np,
                (long long)IB_MAX_POINTS);
  if (!buf->X || !buf->U_prev) return fail(IB_E_INVALID, "null X / U_prev");
  if (!buf->workspace || ((uintptr_t)buf->workspace & 255))
    return fail(IB_E_INVALID, "workspace must be non-null and 256-byte aligned");
  const size_t need = workspace_bytes(prm, np);
  if (buf->workspace_bytes < need)
    return fail(IB_E_INVALID, "workspace too small (%zu < %zu bytes)", buf->workspace_bytes, need);
  if (st->n_links < 0 || (st->n_links > 0 && (!st->a || !st->b || !st->kappa || !st->l0)))
    return fail(IB_E_INVALID, "bad link arrays");
  if (!st->w) return fail(IB_E_INVALID, "null spreading weights");
  for (int64_t i = 0; i < np; i++)
    if (!std::isfinite(st->w[i])) return fail(IB_E_INVALID, "non-finite weight at point %lld", (long long)i);
  if (!st->tether_kappa != !st->tether_target)
    return fail(IB_E_INVALID, "tether stiffness and targets come together (both or neither)");
  if (st->tether_kappa) {
    for (int64_t i = 0; i < np; i++)
      if (!(std::isfinite(st->tether_kappa[i]) && st->tether_kappa[i] >= 0))
        return fail(IB_E_INVALID, "tether stiffness at point %lld must be finite and >= 0", (long long)i);
    for (int64_t i = 0; i < (int64_t)d * np; i++)
      if (!std::isfinite(st->tether_target[i]))
        return fail(IB_E_INVALID, "non-finite tether target (entry %lld)", (long long)i);
  }
  if (st->layer) {
    if (d != 2) return fail(IB_E_INVALID, "point layers are for 2-D batches only");
    for (int64_t i = 0; i < np; i++)
      if (st->layer[i] < 0 || st->layer[i] >= prm->n[2])
        return fail(IB_E_INVALID, "point %lld has layer %d outside [0, %d)", (long long)i,
                    st->layer[i], prm->n[2]);
    for (int64_t e = 0; e < st->n_links; e++)
      if (st->a[e] >= 0 && st->a[e] < np && st->b[e] >= 0 && st->b[e] < np &&
          st->layer[st->a[e]] != st->layer[st->b[e]])
        return fail(IB_E_INVALID, "link %lld joins points of different layers", (long long)e);
  } else if (d == 2 && prm->n[2] > 1) {
    return fail(IB_E_INVALID, "a 2-D batch of %d layers needs the point layers", prm->n[2]);
  }
  // CSR by point, both directions of every link
  std::vector<int32_t> deg(np + 1, 0);
  for (int64_t e = 0; e < st->n_links; e++) {
    const int64_t a = st->a[e], b = st->b[e];
    if (a < 0 || a >= np || b < 0 || b >= np || a == b)
      return fail(IB_E_INVALID, "link %lld has bad endpoints (%lld, %lld)", (long long)e,
                  (long long)a, (long long)b);
    if (!std::isfinite(st->kappa[e]) || !std::isfinite(st->l0[e]) || st->l0[e] < 0)
      return fail(IB_E_INVALID, "link %lld has bad kappa / l0", (long long)e);
    deg[a + 1]++;
    deg[b + 1]++;
  }
  if (2 * st->n_links > INT32_MAX) return fail(IB_E_UNSUPPORTED, "too many links");
  for (int64_t i = 0; i < np; i++) deg[i + 1] += deg[i];
  std::vector<int32_t> nbr(std::max<int64_t>(1, 2 * st->n_links));
  std::vector<double> kap(nbr.size()), l0(nbr.size());
  {
    std::vector<int32_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t e = 0; e < st->n_links; e++) {
      const int32_t a = st->a[e], b = st->b[e];
      int32_t ia = fill[a]++, ib = fill[b]++;
      nbr[ia] = b; kap[ia] = st->kappa[e]; l0[ia] = st->l0[e];
      nbr[ib] = a; kap[ib] = st->kappa[e]; l0[ib] = st->l0[e];
    }
  }
  double ma, mi, pa, pi;
  const double h2 = prm->h * prm->h;
  const double nu = prm->mu * prm->dt / (2.0 * prm->rho);
  if ((s = factor(1.0 + 2.0 * nu / h2, -nu / h2, &ma, &mi)) != IB_OK) return s;
  if ((s = factor(1.0 + 2.0 / h2, -1.0 / h2, &pa, &pi)) != IB_OK) return s;
  const bool layered = d == 2 && (prm->layer_dt || st->layer);
  std::vector<double> l_dt, l_ma, l_mi, l_pi;
  if (layered) {
    for (int l = 0; l < prm->n[2]; l++) {
      const double dtl = prm->layer_dt ? prm->layer_dt[l] : prm->dt;
      const double nul = prm->mu * dtl / (2.0 * prm->rho);
      double a1, i1;
      if ((s = factor(1.0 + 2.0 * nul / h2, -nul / h2, &a1, &i1)) != IB_OK) return s;
      l_dt.push_back(dtl);
      l_ma.push_back(a1);
      l_mi.push_back(i1);
      l_pi.push_back(pi * (-prm->rho / dtl));
    }
  }

  ib_ctx *c = new ib_ctx();
  c->prm = *prm;
  c->buf = *buf;
  c->stream = (hipStream_t)hip_stream;
  c->step = prm->step0;
  c->dim = d;
  c->g.n0 = prm->n[0];
  c->g.n1 = prm->n[1];
  c->g.n2 = prm->n[2];
  c->g.ncell = (int64_t)c->g.n0 * c->g.n1 * c->g.n2;
  c->np = np;
  c->f32 = prm->precision != IB_PREC_FP64;
  c->u64 = prm->precision == IB_PREC_MIXED_STATE64;
  if (prm->dim == 3) {
    // compute units times the workgroups of the 3-D explicit kernel each
    // holds at once (register and LDS limits of this build)
    int dev = 0, ncu = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 1;
    const void *fn = prm->precision == IB_PREC_FP64
                         ? (const void *)k_explicit3<double, double>
                         : (c->u64 ? (const void *)k_explicit3<float, double>
                                   : (const void *)k_explicit3<float, float>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, EX * EY, 0) != hipSuccess) per = 1;
    c->resident3 = std::max(1, ncu) * std::max(1, per);
  }
  c->tsz = c->f32 ? 4 : 8;
  c->mom_alpha = ma; c->mom_invc = mi; c->psi_alpha = pa; c->psi_invc = pi;
  c->nlinks = st->n_links;
  // carve the workspace
  char *w = (char *)buf->workspace;
  const size_t fb = align256((size_t)c->g.ncell * c->tsz);
  const size_t lb = align256(sizeof(double) * d * np);
  for (int i = 0; i < 3; i++) { c->delta[i] = i < d ? (void *)w : nullptr; if (i < d) w += fb; }
  for (int i = 0; i < 3; i++) { c->f[i] = i < d ? (void *)w : nullptr; if (i < d) w += fb; }
  c->divn = w; w += fb;
  c->Xn1 = (double *)w; w += lb;
  c->Xh = (double *)w; w += lb;
  c->F = (double *)w; w += lb;
  c->tg = tile_grid(prm);
  const size_t tb = align256(sizeof(int) * c->tg.ntiles);
  const size_t pb = align256(sizeof(int) * np);
  c->st_x = (double *)w; w += align256(sizeof(double) * 3 * np);
  c->st_val = w; w += align256(c->tsz * 3 * np);
  c->t_count = (int *)w; w += tb;
  c->t_flag = (int *)w; w += tb;
  c->t_list = (int *)w; w += tb;
  c->t_start = (int *)w; w += align256(sizeof(int) * (c->tg.ntiles + 1));
  c->t_bsum = (int *)w; w += align256(sizeof(int) * ((c->tg.ntiles + SCAN_TILE - 1) / SCAN_TILE));
  c->tile_of = (int *)w; w += pb;
  c->rank_of = (int *)w; w += pb;
  c->point_of = (int *)w; w += pb;
  c->t_nlist = (int *)w; w += 256;
  c->flag = (int *)w; w += 256;
  c->gauge = (double *)w;  // [layers] means, then [layers][gauge_blocks] partials
  c->gauge_part = c->gauge + gauge_layers(prm);
  // upload the structure
  auto bail = [&](ib_status e) { ib_destroy(c); return e; };
  // the second stream of the overlapped Lagrangian work (default priority)
  if (hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_u, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_lag, hipEventDisableTiming) != hipSuccess)
    return bail(fail(IB_E_DEVICE, "creating the overlap stream and events failed"));
  if (hipMalloc(&c->ptr, sizeof(int32_t) * (np + 1)) != hipSuccess ||
      hipMalloc(&c->nbr, sizeof(int32_t) * nbr.size()) != hipSuccess ||
      hipMalloc(&c->kap, sizeof(double) * kap.size()) != hipSuccess ||
      hipMalloc(&c->l0, sizeof(double) * l0.size()) != hipSuccess ||
      hipMalloc(&c->w, sizeof(double) * np) != hipSuccess)
    return bail(fail(IB_E_DEVICE, "hipMalloc of the link table failed"));
  if (st->tether_kappa) {
    if (hipMalloc(&c->tk, sizeof(double) * np) != hipSuccess ||
        hipMalloc(&c->ty, sizeof(double) * d * np) != hipSuccess)
      return bail(fail(IB_E_DEVICE, "hipMalloc of the tether table failed"));
    if (hipMemcpy(c->tk, st->tether_kappa, sizeof(double) * np, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->ty, st->tether_target, sizeof(double) * d * np, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(IB_E_DEVICE, "upload of the tether table failed"));
  }
  if (layered) {
    const size_t nl = (size_t)prm->n[2];
    std::vector<int> lay(np, 0);
    if (st->layer)
      for (int64_t i = 0; i < np; i++) lay[i] = st->layer[i];
    if (hipMalloc(&c->p_layer, sizeof(int) * np) != hipSuccess ||
        hipMalloc(&c->l_dt, sizeof(double) * nl) != hipSuccess ||
        hipMalloc(&c->l_mom_alpha, sizeof(double) * nl) != hipSuccess ||
        hipMalloc(&c->l_mom_invc, sizeof(double) * nl) != hipSuccess ||
        hipMalloc(&c->l_psi_invc, sizeof(double) * nl) != hipSuccess)
      return bail(fail(IB_E_DEVICE, "hipMalloc of the layer tables failed"));
    if (hipMemcpy(c->p_layer, lay.data(), sizeof(int) * np, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->l_dt, l_dt.data(), sizeof(double) * nl, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->l_mom_alpha, l_ma.data(), sizeof(double) * nl, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->l_mom_invc, l_mi.data(), sizeof(double) * nl, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->l_psi_invc, l_pi.data(), sizeof(double) * nl, hipMemcpyHostToDevice) != hipSuccess)
      return bail(fail(IB_E_DEVICE, "upload of the layer tables failed"));
  }
  if (hipMemcpyAsync(c->ptr, deg.data(), sizeof(int32_t) * (np + 1), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->nbr, nbr.data(), sizeof(int32_t) * nbr.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->kap, kap.data(), sizeof(double) * kap.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->l0, l0.data(), sizeof(double) * l0.size(), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipMemcpyAsync(c->w, st->w, sizeof(double) * np, hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return bail(fail(IB_E_DEVICE, "upload of the link table failed"));
  // clear the tile counts / flags and the status word; seed div_prev at a
  // fresh start
  if (hipMemsetAsync(c->t_count, 0, tb, c->stream) != hipSuccess ||
      hipMemsetAsync(c->t_flag, 0, tb, c->stream) != hipSuccess ||
      hipMemsetAsync(c->flag, 0, 256, c->stream) != hipSuccess)
    return bail(fail(IB_E_DEVICE, "clearing the workspace failed"));
  if (prm->step0 == 0) seed_divergence(c);
  // the host arrays above go out of scope: wait for the uploads
  if (hipStreamSynchronize(c->stream) != hipSuccess)
    return bail(fail(IB_E_DEVICE, "initialisation on the stream failed"));
  if (hipGetLastError() != hipSuccess) return bail(fail(IB_E_DEVICE, "kernel launch failed"));
  *out = c;
  return IB_OK;
}

extern "C" ib_status ib_restart(ib_ctx *c, int64_t step0) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (step0 < 0) return fail(IB_E_INVALID, "step0 must be >= 0");
  if (c->prof) return fail(IB_E_STATE, "disable profiling before a restart");
  c->step = step0;
  if (step0 == 0) {
    seed_divergence(c);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(IB_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  }
  return IB_OK;
}

extern "C" ib_status ib_refresh_divergence(ib_ctx *c) {
  if (!c) return fail(IB_E_STATE, "null context");
  seed_divergence(c);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IB_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return IB_OK;
}

extern "C" ib_status ib_step(ib_ctx *c, int32_t nsteps) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (nsteps < 0) return fail(IB_E_INVALID, "nsteps < 0");
  for (int32_t i = 0; i < nsteps; i++) enqueue_any(c, i + 1 < nsteps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IB_E_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return IB_OK;
}

// Clear `bytes` (a multiple of 4) with a fill kernel (no memset node).
static void launch_zero_words(void *p, size_t bytes, hipStream_t st) {
  const int64_t n = (int64_t)(bytes / 4);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
  hipLaunchKernelGGL(k_zero_words, dim3(grid), dim3(256), 0, st, (uint32_t *)p, n);
}

// Scan the grid fields (k_field_check) on the context's stream and wait:
// bit 1 of *bad = a velocity component is non-finite, bit 2 = p is; *umax =
// max |u| over all faces.  Uses bytes 8..23 of the status region.
static ib_status check_fields(ib_ctx *c, unsigned *bad, double *umax) {
  unsigned *flags = (unsigned *)((char *)c->flag + 8);
  unsigned long long *bits = (unsigned long long *)((char *)c->flag + 16);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((c->g.ncell + 255) / 256, 2048));
  launch_zero_words(flags, 16, c->stream);
  const double *p = c->buf.p;
  if (c->u64 || !c->f32) {
    const double *u0 = (const double *)c->buf.u[0], *u1 = (const double *)c->buf.u[1],
                 *u2 = (const double *)(c->dim == 3 ? c->buf.u[2] : c->buf.u[0]);
    if (c->dim == 3) hipLaunchKernelGGL((k_field_check<double, 3>), dim3(grid), dim3(256), 0, c->stream, u0, u1, u2, p, c->g.ncell, flags, bits);
    else hipLaunchKernelGGL((k_field_check<double, 2>), dim3(grid), dim3(256), 0, c->stream, u0, u1, u2, p, c->g.ncell, flags, bits);
  } else {
    const float *u0 = (const float *)c->buf.u[0], *u1 = (const float *)c->buf.u[1],
                *u2 = (const float *)(c->dim == 3 ? c->buf.u[2] : c->buf.u[0]);
    if (c->dim == 3) hipLaunchKernelGGL((k_field_check<float, 3>), dim3(grid), dim3(256), 0, c->stream, u0, u1, u2, p, c->g.ncell, flags, bits);
    else hipLaunchKernelGGL((k_field_check<float, 2>), dim3(grid), dim3(256), 0, c->stream, u0, u1, u2, p, c->g.ncell, flags, bits);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(c->stream));
  unsigned long long host[2] = {0, 0};
  HIP_TRY(hipMemcpy(host, (char *)c->flag + 8, 16, hipMemcpyDeviceToHost));
  *bad = (unsigned)(host[0] & 0xffffffffu);
  double m;
  std::memcpy(&m, &host[1], sizeof(double));
  *umax = m;
  return IB_OK;
}

static ib_status nonfinite_fields(const ib_ctx *c, unsigned bad) {
  return fail(IB_E_NONFINITE, "%s%s%s became non-finite (step <= %lld)",
              (bad & 1u) ? "the velocity u" : "", (bad & 3u) == 3u ? " and " : "",
              (bad & 2u) ? "the pressure p" : "", (long long)c->step);
}

extern "C" ib_status ib_sync(ib_ctx *c, int64_t *step_index) {
  if (!c) return fail(IB_E_STATE, "null context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (step_index) *step_index = c->step;
  int flag = 0;
  HIP_TRY(hipMemcpy(&flag, c->flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) return fail(IB_E_NONFINITE, "a Lagrangian position became non-finite (step <= %lld)",
                        (long long)c->step);
  unsigned bad = 0;
  double umax = 0.0;
  ib_status s = check_fields(c, &bad, &umax);
  if (s != IB_OK) return s;
  if (bad) return nonfinite_fields(c, bad);
  return IB_OK;
}

extern "C" ib_status ib_check_fields(ib_ctx *c, double *max_abs_u) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (!max_abs_u) return fail(IB_E_INVALID, "null output");
  unsigned bad = 0;
  ib_status s = check_fields(c, &bad, max_abs_u);
  if (s != IB_OK) return s;
  if (bad) return nonfinite_fields(c, bad);
  return IB_OK;
}

extern "C" ib_status ib_spread(ib_ctx *c, const double *X, const double *F, const double *w,
                               int64_t npts, void *const f_out[3], int32_t accumulate) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (npts < 0 || (npts > 0 && (!X || !F || !w)) || !f_out)
    return fail(IB_E_INVALID, "bad spread arguments");
  if (npts > c->np)
    return fail(IB_E_INVALID, "npts %lld exceeds the context's %lld points", (long long)npts,
                (long long)c->np);
  for (int i = 0; i < c->dim; i++)
    if (!f_out[i]) return fail(IB_E_INVALID, "null output component %d", i);
  if (!accumulate)
    for (int i = 0; i < c->dim; i++)
      HIP_TRY(hipMemsetAsync(f_out[i], 0, (size_t)c->g.ncell * c->tsz, c->stream));
  if (npts == 0) return IB_OK;
  if (c->f32) {
    if (c->dim == 2) launch_spread<float, 2, true>(c, X, F, w, npts, f_out);
    else launch_spread<float, 3, true>(c, X, F, w, npts, f_out);
  } else {
    if (c->dim == 2) launch_spread<double, 2, true>(c, X, F, w, npts, f_out);
    else launch_spread<double, 3, true>(c, X, F, w, npts, f_out);
  }
  HIP_TRY(hipGetLastError());
  return IB_OK;
}

// ------------------------------------------- spreading without allocation --

// The scratch of ib_spread_static: one fixed device array, a copy per GPU
// that the library runs on, held until the process ends.  In host code the
// name `scratch` is only a stand-in for the symbol (passing it to a kernel
// would hand the device a host address): its device address is looked up
// once per device, with that device current, and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[IB_SPREAD_STATIC_MAX_BYTES];
constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_dev[kScratchDevices];

static ib_status scratch_of_current_device(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kScratchDevices)
    return fail(IB_E_UNSUPPORTED, "device %d: the static spreading scratch tracks devices 0..%d",
                dev, kScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(IB_E_DEVICE, "hipGetSymbolAddress of the spreading scratch failed: %s",
                  hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return IB_OK;
}

// Spreading tables of `np` points on the grid of `p`, carved from `base`
// (or counted, with base = nullptr): the sorted stencils (start cells,
// weights, values), the tile counts, list and starts, the block sums of the
// scan, the point sort (tile, rank) and the list length.
static size_t carve_spread_tables(ib_ctx *c, const ib_grid_params *p, int64_t np, char *base) {
  const size_t t = p->precision == IB_PREC_FP64 ? 8 : 4;
  const size_t npp = (size_t)(np > 0 ? np : 1);
  const TileGrid tg = tile_grid(p);
  const size_t tb = align256(sizeof(int) * (size_t)tg.ntiles);
  const size_t pb = align256(sizeof(int) * npp);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    void *q = base ? (void *)(base + off) : nullptr;
    off += bytes;
    return q;
  };
  void *st_x = take(align256(sizeof(double) * 3 * npp));
  void *st_val = take(align256(t * 3 * npp));
  void *t_count = take(tb);
  void *t_list = take(tb);
  void *t_start = take(align256(sizeof(int) * (size_t)(tg.ntiles + 1)));
  void *t_bsum = take(align256(sizeof(int) * (size_t)((tg.ntiles + SCAN_TILE - 1) / SCAN_TILE)));
  void *tile_of = take(pb);
  void *rank_of = take(pb);
  void *point_of = take(pb);
  void *t_nlist = take(256);
  if (c) {
    c->tg = tg;
    c->st_x = (double *)st_x;
    c->st_val = st_val;
    c->t_count = (int *)t_count;
    c->t_list = (int *)t_list;
    c->t_start = (int *)t_start;
    c->t_bsum = (int *)t_bsum;
    c->tile_of = (int *)tile_of;
    c->rank_of = (int *)rank_of;
    c->point_of = (int *)point_of;
    c->t_nlist = (int *)t_nlist;
  }
  return off;
}

extern "C" ib_status ib_spread_static(const ib_grid_params *prm, const double *X, const double *F,
                                      const double *w, int64_t npts, void *const f_out[3],
                                      int32_t accumulate, void *hip_stream) {
  ib_status s = check_params(prm);
  if (s != IB_OK) return s;
  if (prm->dim == 2 && prm->n[2] != 1)
    return fail(IB_E_INVALID, "ib_spread_static takes one 2-D problem (n[2] = 1), not a batch");
  if (npts < 0 || (npts > 0 && (!X || !F || !w)) || !f_out)
    return fail(IB_E_INVALID, "bad spread arguments");
  for (int i = 0; i < prm->dim; i++)
    if (!f_out[i]) return fail(IB_E_INVALID, "null output component %d", i);
  if (npts > IB_MAX_POINTS)
    return fail(IB_E_UNSUPPORTED, "npts above IB_MAX_POINTS (32-bit sort ranks)");
  const size_t need = carve_spread_tables(nullptr, prm, npts, nullptr);
  if (need > (size_t)IB_SPREAD_STATIC_MAX_BYTES)
    return fail(IB_E_UNSUPPORTED,
                "%lld points on this grid need %zu bytes of spreading scratch, above the %zu "
                "bytes of the static array (use ib_spread with a workspace)",
                (long long)npts, need, (size_t)IB_SPREAD_STATIC_MAX_BYTES);
  void *base = nullptr;
  if ((s = scratch_of_current_device(&base)) != IB_OK) return s;
  // a host-side description of the grid and the tables (no allocation)
  ib_ctx c{};
  c.prm = *prm;
  c.stream = (hipStream_t)hip_stream;
  c.dim = prm->dim;
  c.g.n0 = prm->n[0];
  c.g.n1 = prm->n[1];
  c.g.n2 = prm->n[2];
  c.g.ncell = (int64_t)c.g.n0 * c.g.n1 * c.g.n2;
  c.f32 = prm->precision != IB_PREC_FP64;
  c.tsz = c.f32 ? 4 : 8;
  carve_spread_tables(&c, prm, npts, (char *)base);
  // the array keeps the last call's contents: clear the tile counts (the
  // binning counts with atomics) and, unless accumulating, the output
  launch_zero_words(c.t_count, sizeof(int) * (size_t)c.tg.ntiles, c.stream);
  if (!accumulate)
    for (int i = 0; i < c.dim; i++) launch_zero_words(f_out[i], (size_t)c.g.ncell * c.tsz, c.stream);
  if (npts > 0) {
    if (c.f32) {
      if (c.dim == 2) launch_spread<float, 2, true>(&c, X, F, w, npts, f_out);
      else launch_spread<float, 3, true>(&c, X, F, w, npts, f_out);
    } else {
      if (c.dim == 2) launch_spread<double, 2, true>(&c, X, F, w, npts, f_out);
      else launch_spread<double, 3, true>(&c, X, F, w, npts, f_out);
    }
  }
  HIP_TRY(hipGetLastError());
  return IB_OK;
}

template <typename T, int DIM>
static void launch_force_dense(ib_ctx *c, void *const f_out[3]) {
  const unsigned nb = (unsigned)((c->g.ncell + 255) / 256);
  k_force_dense<T, DIM><<<nb, 256, 0, c->stream>>>(
      (const T *)c->f[0], (const T *)c->f[1], (const T *)(DIM == 3 ? c->f[2] : c->f[0]),
      c->t_flag, c->g, c->tg, (T *)f_out[0], (T *)f_out[1], (T *)(DIM == 3 ? f_out[2] : f_out[0]));
}

extern "C" ib_status ib_step_force(ib_ctx *c, void *const f_out[3]) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (!c->have_force) return fail(IB_E_STATE, "no step has been taken yet");
  if (!f_out) return fail(IB_E_INVALID, "null output");
  for (int i = 0; i < c->dim; i++)
    if (!f_out[i]) return fail(IB_E_INVALID, "null output component %d", i);
  if (c->f32) {
    if (c->dim == 2) launch_force_dense<float, 2>(c, f_out);
    else launch_force_dense<float, 3>(c, f_out);
  } else {
    if (c->dim == 2) launch_force_dense<double, 2>(c, f_out);
    else launch_force_dense<double, 3>(c, f_out);
  }
  HIP_TRY(hipGetLastError());
  return IB_OK;
}

extern "C" ib_status ib_interp(ib_ctx *c, const double *X, int64_t npts, void *const u_in[3],
                               double *U) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (npts < 0 || (npts > 0 && (!X || !U)) || !u_in)
    return fail(IB_E_INVALID, "bad interp arguments");
  if (c->p_layer && npts > c->np)
    return fail(IB_E_INVALID, "npts %lld exceeds the batch's %lld points", (long long)npts,
                (long long)c->np);
  for (int i = 0; i < c->dim; i++)
    if (!u_in[i]) return fail(IB_E_INVALID, "null input component %d", i);
  if (npts == 0) return IB_OK;
  if (c->f32 && !c->u64) {
    if (c->dim == 2) launch_interp<float, 2>(c, KP_INTERP, X, npts, u_in, U, false, false);
    else launch_interp<float, 3>(c, KP_INTERP, X, npts, u_in, U, false, false);
  } else {
    if (c->dim == 2) launch_interp<double, 2>(c, KP_INTERP, X, npts, u_in, U, false, false);
    else launch_interp<double, 3>(c, KP_INTERP, X, npts, u_in, U, false, false);
  }
  HIP_TRY(hipGetLastError());
  return IB_OK;
}

extern "C" ib_status ib_force(ib_ctx *c, const double *X, double *F) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (!X || !F) return fail(IB_E_INVALID, "bad force arguments");
  if (c->dim == 2) launch_force<2>(c, X, F, false);
  else launch_force<3>(c, X, F, false);
  HIP_TRY(hipGetLastError());
  return IB_OK;
}

extern "C" ib_status ib_line_solve(void *data, int32_t dtype, const int32_t n[3], int32_t axis,
                                   int32_t nfields, int64_t field_stride, double diag,
                                   double off, void *hip_stream) {
  if (!data || !n) return fail(IB_E_INVALID, "null data / shape");
  if (dtype != IB_F64 && dtype != IB_F32) return fail(IB_E_INVALID, "unknown dtype %d", dtype);
  if (axis < 0 || axis > 2) return fail(IB_E_INVALID, "axis must be 0, 1 or 2");
  for (int a = 0; a < 3; a++)
    if (n[a] < 1) return fail(IB_E_INVALID, "n[%d] < 1", a);
  if (n[axis] < 3) return fail(IB_E_INVALID, "lines must have >= 3 points");
  if (n[axis] > 1024) return fail(IB_E_UNSUPPORTED, "lines longer than 1024 are not built");
  if (n[0] > 65535 * 64LL || (int64_t)n[1] * n[2] > ((int64_t)1 << 40))
    return fail(IB_E_UNSUPPORTED, "array too large");
  if (nfields < 1) return fail(IB_E_INVALID, "nfields < 1");
  const int64_t ncell = (int64_t)n[0] * n[1] * n[2];
  if (nfields > 1 && field_stride < ncell)
    return fail(IB_E_INVALID, "field_stride < n0 n1 n2 would overlap fields");
  double al, ic;
  ib_status s = factor(diag, off, &al, &ic);
  if (s != IB_OK) return s;
  hipStream_t st = (hipStream_t)hip_stream;
  Grid g{n[0], n[1], n[2], ncell};
  for (int f0 = 0; f0 < nfields; f0 += 3) {
    const int nf = std::min(3, nfields - f0);
    if (dtype == IB_F64) {
      SweepArgs<double> a{};
      a.g = g; a.alpha = al; a.inv_c = ic;
      for (int i = 0; i < nf; i++) a.f[i] = a.o[i] = (double *)data + (f0 + i) * field_stride;
      sweep<double, SW_PLAIN>(nullptr, KP_LINE_X, a, axis, nf, st);
    } else {
      SweepArgs<float> a{};
      a.g = g; a.alpha = al; a.inv_c = ic;
      for (int i = 0; i < nf; i++) a.f[i] = a.o[i] = (float *)data + (f0 + i) * field_stride;
      sweep<float, SW_PLAIN>(nullptr, KP_LINE_X, a, axis, nf, st);
    }
  }
  HIP_TRY(hipGetLastError());
  return IB_OK;
}

extern "C" ib_status ib_destroy(ib_ctx *c) {
  if (!c) return IB_OK;
  (void)hipStreamSynchronize(c->stream);
  for (auto &p : c->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : c->pool) (void)hipEventDestroy(e);
  if (c->ptr) (void)hipFree(c->ptr);
  if (c->nbr) (void)hipFree(c->nbr);
  if (c->kap) (void)hipFree(c->kap);
  if (c->l0) (void)hipFree(c->l0);
  if (c->w) (void)hipFree(c->w);
  if (c->tk) (void)hipFree(c->tk);
  if (c->ty) (void)hipFree(c->ty);
  if (c->stream2) {
    (void)hipStreamSynchronize(c->stream2);
    (void)hipStreamDestroy(c->stream2);
  }
  if (c->ev_u) (void)hipEventDestroy(c->ev_u);
  if (c->ev_lag) (void)hipEventDestroy(c->ev_lag);
  for (void *q : {(void *)c->p_layer, (void *)c->l_dt, (void *)c->l_mom_alpha,
                  (void *)c->l_mom_invc, (void *)c->l_psi_invc})
    if (q) (void)hipFree(q);
  delete c;
  return IB_OK;
}

extern "C" ib_status ib_profile_enable(ib_ctx *c, int32_t enable) {
  if (!c) return fail(IB_E_STATE, "null context");
  HIP_TRY(hipStreamSynchronize(c->stream));
  drain_events(c);
  for (int i = 0; i < KP_COUNT; i++) {
    c->prof_ms[i] = 0;
    c->prof_n[i] = 0;
  }
  c->prof = enable != 0;
  return IB_OK;
}

extern "C" int32_t ib_profile_count(void) { return KP_COUNT; }

extern "C" const char *ib_profile_name(int32_t id) {
  return (id >= 0 && id < KP_COUNT) ? kKernelNames[id] : "";
}

extern "C" ib_status ib_profile_read(ib_ctx *c, int32_t id, double *total_ms,
                                     int64_t *launches) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (id < 0 || id >= KP_COUNT) return fail(IB_E_INVALID, "kernel id out of range");
  drain_events(c);
  if (total_ms) *total_ms = c->prof_ms[id];
  if (launches) *launches = c->prof_n[id];
  return IB_OK;
}

// ----------------------------------------------------------- autotuner --

static void enqueue_any(ib_ctx *c, bool overlap) {
  if (c->u64) {
    if (c->dim == 2) enqueue_step<float, 2, double>(c, overlap);
    else enqueue_step<float, 3, double>(c, overlap);
  } else if (c->f32) {
    if (c->dim == 2) enqueue_step<float, 2, float>(c, overlap);
    else enqueue_step<float, 3, float>(c, overlap);
  } else {
    if (c->dim == 2) enqueue_step<double, 2, double>(c, overlap);
    else enqueue_step<double, 3, double>(c, overlap);
  }
}

static int x_chunk64(int64_t N) {
  static const int ms[] = {1, 2, 4, 6, 8, 12, 16, 32};
  for (int m : ms)
    if ((N + m - 1) / m <= 64) return m;
  return 32;
}

// Time one plain sweep configuration `reps` times on the context's scratch
// fields (the momentum increments, free outside a step).
template <typename T, typename R>
static float time_sweep(ib_ctx *c, int axis, int nf, const SweepTune &tu, int reps,
                        hipEvent_t e0, hipEvent_t e1) {
  SweepArgs<T> a{};
  a.g = c->g;
  a.dim = c->dim;
  a.alpha = c->psi_alpha;
  a.inv_c = c->psi_invc;
  for (int i = 0; i < nf; i++) a.f[i] = a.o[i] = (T *)c->delta[i];
  auto run = [&] {
    if (axis == 0) dispatch_x<T, SW_PLAIN>(a, nf, c->stream, &tu);
    else dispatch_s<T, SW_PLAIN, R>(a, axis, nf, c->stream, &tu);
  };
  run();
  (void)hipEventRecord(e0, c->stream);
  for (int r = 0; r < reps; r++) run();
  (void)hipEventRecord(e1, c->stream);
  (void)hipEventSynchronize(e1);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  return ms;
}

template <typename T>
static void tune_ctx(ib_ctx *c, int reps, hipEvent_t e0, hipEvent_t e1) {
  const int nn[3] = {c->g.n0, c->g.n1, c->g.n2};
  for (int axis = 0; axis < c->dim; axis++) {
    const int64_t N = nn[axis];
    for (int r64 = 0; r64 < 2; r64++) {
      // the mixed policy runs momentum (all components) with FP32 recurrences
      // and psi (one field) with FP64 ones; FP64 runs everything in FP64
      const bool rd = r64 || !c->f32;
      const int nf = (c->f32 && r64) ? 1 : c->dim;
      std::vector<SweepTune> cand;
      if (axis == 0) {
        cand.push_back({x_chunk(N), 0, 0});
        if (x_chunk64(N) != x_chunk(N)) cand.push_back({x_chunk64(N), 0, 0});
      } else {
        for (int m : {16, 32})
          for (int tx : {32, 64})
            if (tx * ((N + m - 1) / m) <= 1024) cand.push_back({0, tx, m});
      }
      float best = 1e30f;
      SweepTune pick = cand.empty() ? SweepTune{0, 0, 0} : cand[0];
      for (const SweepTune &t : cand) {
        const float ms = rd ? time_sweep<T, double>(c, axis, nf, t, reps, e0, e1)
                            : time_sweep<T, float>(c, axis, nf, t, reps, e0, e1);
        if (ms < best) {
          best = ms;
          pick = t;
        }
      }
      c->tune[axis][r64] = pick;
    }
  }
}

extern "C" ib_status ib_tune(ib_ctx *c, int32_t reps) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (c->prof) return fail(IB_E_STATE, "disable profiling before tuning");
  if (reps < 1 || reps > 1000) return fail(IB_E_INVALID, "reps must lie in [1, 1000]");
  HIP_TRY(hipStreamSynchronize(c->stream));
  const size_t fb = align256((size_t)c->g.ncell * c->tsz);
  for (int i = 0; i < c->dim; i++) HIP_TRY(hipMemsetAsync(c->delta[i], 0, fb, c->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(IB_E_DEVICE, "hipEventCreate failed");
  }
  c->tuned = false;
  if (c->f32) tune_ctx<float>(c, reps, e0, e1);
  else tune_ctx<double>(c, reps, e0, e1);
  c->tuned = true;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(IB_E_DEVICE, "tuning launch failed: %s", hipGetErrorString(e));
  return IB_OK;
}

extern "C" ib_status ib_tune_read(const ib_ctx *c, int32_t axis, int32_t fp64_recurrence,
                                  int32_t *x_chunk_out, int32_t *s_rows_out,
                                  int32_t *s_chunk_out) {
  if (!c) return fail(IB_E_STATE, "null context");
  if (axis < 0 || axis >= c->dim) return fail(IB_E_INVALID, "axis out of range");
  const SweepTune t = c->tuned ? c->tune[axis][fp64_recurrence ? 1 : 0] : SweepTune{0, 0, 0};
  if (x_chunk_out) *x_chunk_out = t.x_m;
  if (s_rows_out) *s_rows_out = t.s_tx;
  if (s_chunk_out) *s_chunk_out = t.s_m;
  return IB_OK;
}

// ---------------------------------------------------------- graph launch --

struct ib_graph {
  std::vector<ib_ctx *> ctx;
  int spl;
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

// Capture `spl` steps of every context.  Without IB_GRAPH_BRANCHES the graph
// is one chain (step s of every context, then step s + 1).  With it, each
// context is recorded on a stream of its own forked from `st` and joined back,
// so the graph holds one independent branch per context, which the runtime may
// run concurrently (the problems share no data).
// (Captured steps do not overlap the next step's Lagrangian work on the
// context's second stream: a capture holding that fork and join ended in a
// crash inside the runtime.  Graphs of several contexts overlap through their
// branches instead.)
static ib_status capture_steps(ib_ctx *const *ctxs, int32_t nctx, int32_t spl, hipStream_t st,
                               int32_t flags, hipGraph_t *graph) {
  const bool branches = (flags & IB_GRAPH_BRANCHES) && nctx > 1;
  std::vector<hipStream_t> br;
  std::vector<hipEvent_t> ev;
  auto cleanup = [&]() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    for (hipStream_t b : br) (void)hipStreamDestroy(b);
  };
  if (branches) {
    br.resize(nctx, nullptr);
    ev.resize(nctx + 1, nullptr);
    for (int i = 0; i < nctx; i++)
      if (hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking) != hipSuccess) {
        cleanup();
        return fail(IB_E_DEVICE, "hipStreamCreateWithFlags failed");
      }
    for (int i = 0; i <= nctx; i++)
      if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) {
        cleanup();
        return fail(IB_E_DEVICE, "hipEventCreateWithFlags failed");
      }
  }
  std::vector<int64_t> saved(nctx);
  std::vector<hipStream_t> own(nctx);
  for (int i = 0; i < nctx; i++) saved[i] = ctxs[i]->step, own[i] = ctxs[i]->stream;
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    cleanup();
    return fail(IB_E_DEVICE, "hipStreamBeginCapture failed: %s", hipGetErrorString(e));
  }
  hipError_t ef = hipSuccess;
  if (branches) {
    ef = hipEventRecord(ev[nctx], st);
    for (int i = 0; i < nctx && ef == hipSuccess; i++) {
      ef = hipStreamWaitEvent(br[i], ev[nctx], 0);
      ctxs[i]->stream = br[i];
      for (int k = 0; k < spl && ef == hipSuccess; k++) enqueue_any(ctxs[i], false);
      if (ef == hipSuccess) ef = hipEventRecord(ev[i], br[i]);
      if (ef == hipSuccess) ef = hipStreamWaitEvent(st, ev[i], 0);
    }
  } else {
    for (int k = 0; k < spl; k++)
      for (int i = 0; i < nctx; i++) enqueue_any(ctxs[i], false);
  }
  hipError_t el = hipGetLastError();
  e = hipStreamEndCapture(st, graph);
  for (int i = 0; i < nctx; i++) ctxs[i]->step = saved[i], ctxs[i]->stream = own[i];
  cleanup();
  if (ef != hipSuccess)
    return fail(IB_E_DEVICE, "fork/join during capture failed: %s", hipGetErrorString(ef));
  if (el != hipSuccess)
    return fail(IB_E_DEVICE, "kernel launch during capture failed: %s", hipGetErrorString(el));
  if (e != hipSuccess || !*graph)
    return fail(IB_E_DEVICE, "stream capture failed: %s", hipGetErrorString(e));
  return IB_OK;
}

extern "C" ib_status ib_graph_create(ib_graph **out, ib_ctx *const *ctxs, int32_t nctx,
                                     int32_t steps_per_launch, int32_t flags, void *hip_stream) {
  if (!out) return fail(IB_E_INVALID, "null graph output");
  *out = nullptr;
  if (!ctxs || nctx < 1) return fail(IB_E_INVALID, "no contexts");
  if (steps_per_launch < 1) return fail(IB_E_INVALID, "steps_per_launch < 1");
  if (flags & ~IB_GRAPH_BRANCHES) return fail(IB_E_INVALID, "unknown graph flags %d", flags);
  hipStream_t st = (hipStream_t)hip_stream;
  if (!st) return fail(IB_E_INVALID, "graph capture needs a created stream, not the null stream");
  for (int i = 0; i < nctx; i++) {
    ib_ctx *c = ctxs[i];
    if (!c) return fail(IB_E_INVALID, "null context %d", i);
    for (int j = 0; j < i; j++)
      if (ctxs[j] == c) return fail(IB_E_INVALID, "context %d listed twice", i);
    if (c->stream != st) return fail(IB_E_INVALID, "context %d uses another stream", i);
    if (c->prof) return fail(IB_E_STATE, "context %d is profiling", i);
    if (c->step < 1)
      return fail(IB_E_STATE, "context %d is at step 0: take the first step with ib_step", i);
    const int period = c->prm.rotate_split ? c->dim : 1;
    if (steps_per_launch % period != 0)
      return fail(IB_E_INVALID, "steps_per_launch must be a multiple of %d (context %d)",
                  period, i);
  }
  HIP_TRY(hipStreamSynchronize(st));
  hipGraph_t graph = nullptr;
  ib_status s = capture_steps(ctxs, nctx, steps_per_launch, st, flags, &graph);
  if (s != IB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return fail(IB_E_DEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  ib_graph *g = new ib_graph();
  g->ctx.assign(ctxs, ctxs + nctx);
  g->spl = steps_per_launch;
  g->stream = st;
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return IB_OK;
}

extern "C" ib_status ib_graph_launch(ib_graph *g, int32_t nlaunches) {
  if (!g) return fail(IB_E_STATE, "null graph");
  if (nlaunches < 0) return fail(IB_E_INVALID, "nlaunches < 0");
  for (int32_t i = 0; i < nlaunches; i++) {
    HIP_TRY(hipGraphLaunch(g->exec, g->stream));
    for (ib_ctx *c : g->ctx) c->step += g->spl;
  }
  return IB_OK;
}

extern "C" ib_status ib_graph_destroy(ib_graph *g) {
  if (!g) return IB_OK;
  (void)hipStreamSynchronize(g->stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return IB_OK;
}
