/*
 * ibgm.h -- C ABI of libibgm.so, the MI355X (gfx950) IB-GM time-step library.
 *
 * The method is the immersed-boundary algorithm built on the Guermond-Minev
 * direction-split, pseudo-compressible Navier-Stokes solver of Wiens &
 * Stockie ("An efficient parallel immersed boundary algorithm using a
 * pseudo-compressible fluid solver"): a periodic box of side n[a]*h, constant
 * density rho and viscosity mu, a MAC (staggered) grid, Lagrangian points
 * joined by elastic links, a fixed time step dt (Sec. "Immersed Boundary
 * Equations", Sec. "Discretization of Fluid and IB Domains").
 *
 * Conventions shared by every entry point
 *   Pointers.   Every array argument is a DEVICE pointer (hipMalloc / torch
 *               CUDA tensor) unless the comment says "host".  The caller
 *               owns every buffer; the library never frees caller memory.
 *   Layout.     Grid arrays are dense [n2][n1][n0] (x fastest; in 2D, n2 is
 *               the number of independent layers, 1 for one problem).
 *               Velocity component c lives on the faces normal to axis c:
 *               integer index along c, half-integer along the others; cell
 *               centred arrays (p, psi, div) sit at half-integers.  Lagrangian
 *               arrays are structure-of-arrays [dim][n_points] FP64, with
 *               positions unwrapped (grid indices are taken mod n).
 *   Precision.  IB_PREC_FP64: every grid array is FP64.  IB_PREC_MIXED: the
 *               velocity-like grid arrays (u, nl_prev, psi, div_prev, the
 *               workspace and spread forces) are FP32, while p, X, U stay
 *               FP64.  IB_PREC_MIXED_STATE64: as MIXED, but the velocity u
 *               is FP64 (the explicit step computes in FP64, the momentum
 *               sweeps solve FP32 increments, u += increment in FP64), which
 *               keeps D.u^{n+1} -- and so psi and p -- free of the FP32
 *               rounding of u.  "grid dtype" below is FP32 for both mixed
 *               policies; u_in of ib_interp and the u buffers take the
 *               velocity dtype.  Pressure-increment recurrences always run in
 *               FP64 registers; momentum recurrences in the storage
 *               precision.
 *   Streams.    Work is enqueued on the hipStream_t given to ib_init (or to
 *               ib_line_solve) and returns before it completes.  Device faults
 *               surface at the next call that synchronises (ib_sync).
 *   Errors.     Every call returns an ib_status.  IB_E_INVALID means nothing
 *               was enqueued and no state changed; ib_last_error() holds a
 *               message for the calling thread.  No C++ exception crosses
 *               this boundary.  One ib_ctx is used by one host thread at a
 *               time.
 */
#ifndef IBGM_H
#define IBGM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ib_ctx ib_ctx;

typedef enum {
  IB_OK = 0,
  IB_E_INVALID = 1,     /* bad argument; nothing enqueued */
  IB_E_UNSUPPORTED = 2, /* valid but not built (e.g. a line longer than 1024) */
  IB_E_DEVICE = 3,      /* a HIP runtime call failed */
  IB_E_NONFINITE = 4,   /* a Lagrangian position became NaN/Inf (ib_sync) */
  IB_E_STATE = 5        /* call out of order (e.g. null context) */
} ib_status;

typedef enum { IB_F64 = 0, IB_F32 = 1 } ib_dtype;
typedef enum {
  IB_PREC_FP64 = 0,         /* every grid array FP64 */
  IB_PREC_MIXED = 1,        /* FP32 grid arrays; FP64 p, X, U */
  IB_PREC_MIXED_STATE64 = 2 /* FP32 line solves, spreading and work arrays
                               (nl_prev, psi, div_prev, workspace); FP64
                               velocity u, p, X, U */
} ib_precision;

/* flags */
#define IB_FLAG_NO_ADVECTION 1 /* drop the advection term (Stokes flow) */
/* No-slip walls at y = 0 and y = n[1] h: a channel, periodic in x (and z).
 * The solver is not tied to periodic boundaries and the channel is the
 * paper's example (Sec. "Comparison with Poisson Solvers").  u (and w) take
 * the ghost value -u across a wall (2 U - u across the upper wall when it
 * moves with U, ib_grid_params.wall_velocity), v is zero on the wall faces (y-face row
 * j = 0, which is both walls periodically; the caller's initial v must be
 * zero there), psi takes a homogeneous Neumann condition; the y sweeps solve
 * these bounded systems as periodic ones on the odd / even mirror image of
 * each line.  Requires 32 <= n[1] <= 512 with n[1] a multiple of 16 (of 32
 * above 256).  Lagrangian points must stay at least 2h from the walls (the
 * 4-point stencils then never reach across them); nothing checks this. */
#define IB_FLAG_WALLS_Y 2
/* Deterministic spreading (Step 2b): the points of each spreading tile are
 * put in point-index order and every grid cell adds its contributions in one
 * fixed order without atomics, so every step -- and a restart from a saved
 * state -- is bitwise reproducible run to run.  Slower spreading (each cell
 * visits every candidate point of its tile); for verification, not speed.
 * Without it the sums are formed with atomics and their last bits vary. */
#define IB_FLAG_DETERMINISTIC_SPREAD 4

/* Largest number of immersed points per context: points are sorted by tile
 * with 32-bit counts and ranks. */
#define IB_MAX_POINTS 2147483647LL

typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t n[3];         /* cells per axis, each >= 4 and <= 1024.  In 2D, n[2]
                           counts independent layers: n[2] equal-size 2-D
                           problems stacked along the slowest axis, never
                           coupled (a batch; 1 for a single problem) */
  double h;             /* mesh width > 0 (the paper's h = H/N) */
  double rho;           /* density > 0 */
  double mu;            /* dynamic viscosity >= 0 */
  double dt;            /* time step > 0; the pseudo-compressibility eps = dt */
  double chi;           /* pressure-correction weight chi in (0, 1]; 0.6 in the paper */
  int32_t precision;    /* ib_precision */
  int32_t rotate_split; /* 1: rotate the split order every step (Sec.
                           "Partitioning of the Eulerian and Lagrangian Grids",
                           GM modifications); step n uses the n-th cyclic shift
                           of (x, y[, z]) for momentum and psi sweeps alike */
  int32_t flags;        /* IB_FLAG_* */
  int64_t step0;        /* index n of the state handed in; 0 = fresh start, which
                           applies the paper's n = 0 rules (forward Euler for X,
                           N^{1/2} = N(u^0)) and computes div_prev = D.u^0 */
  const double *layer_dt; /* HOST, 2-D batches: time step of each of the n[2]
                           layers (each > 0), or NULL for dt everywhere;
                           copied at ib_init */
  double body_force[3]; /* uniform force density g added to the fluid force f
                           of the momentum equation (Sec. "Governing
                           Equations"), e.g. the mean pressure gradient that
                           drives a channel; zeros for none; finite */
  double wall_velocity[3]; /* IB_FLAG_WALLS_Y: velocity of the upper wall
                           (y = n[1] h), tangential only ([0], and [2] in
                           3-D; [1] must be 0); the lower wall is at rest.
                           Across it a tangential component takes the ghost
                           2 U - u.  A moving wall drives Couette flow.  Zeros
                           without walls (else IB_E_INVALID); finite */
} ib_grid_params;

/* Device state, caller-owned, borrowed by the context until ib_destroy.
 * "grid dtype" = FP64 (IB_PREC_FP64) or FP32 (IB_PREC_MIXED). */
typedef struct {
  void *u[3];       /* u^n per component, velocity dtype, [n2][n1][n0]; updated in place */
  void *nl_prev[3]; /* N(u^{n-1}) (skew advection), grid dtype; overwritten each step */
  void *psi;        /* psi^{n-1/2}, grid dtype, cell centred */
  void *div_prev;   /* D.u^n, grid dtype, cell centred (written by ib_init if step0 == 0) */
  double *p;        /* p^{n-1/2}, FP64, cell centred */
  double *X;        /* X^n, FP64 [dim][n_points] */
  double *U_prev;   /* U^{n-1}, FP64 [dim][n_points] */
  int64_t n_points; /* 1 .. IB_MAX_POINTS (larger: IB_E_UNSUPPORTED) */
  void *workspace;  /* device scratch of ib_workspace_size() bytes, 256-B aligned */
  size_t workspace_bytes;
} ib_buffers;

/* Elastic structure: HOST arrays, copied at ib_init (force-connection form of
 * Step 2a: link e pulls a[e], b[e] together with
 * kappa[e] (X_b - X_a)(1 - l0[e]/|X_b - X_a|); a fiber of the paper with
 * stiffness sigma, rest strain L and spacing h_s has kappa = sigma/h_s^2,
 * l0 = L h_s and spreading weight w = h_s).  X_b - X_a is the nearest
 * periodic image in the box [0, n[c] h): a fiber may close through its
 * periodic copy, as the axial fibers of the cylinder of Sec. "Cylindrical
 * Shell in 3D" do; a link must be shorter than half the box. */
typedef struct {
  int64_t n_links;
  const int32_t *a, *b;      /* host, point indices in [0, n_points) */
  const double *kappa, *l0;  /* host, kappa finite, l0 >= 0 */
  const double *w;           /* host [n_points], spreading weight (Step 2b) */
  const int32_t *layer;      /* host [n_points], 2-D batches: the layer (in
                                [0, n[2])) each point lives in, or NULL for 0;
                                links must not join points of different layers */
  /* Tether points (Sec. "Introduction to the GM method": complex solid
   * boundaries as immersed points attached to fixed tether points): point k
   * feels kappa_t[k] (Y_k - X_k) towards its fixed target Y_k (nearest
   * periodic image), added to its link force in Step 2a.  Both NULL: no
   * tethers. */
  const double *tether_kappa;  /* host [n_points], >= 0 (0: point not tethered) */
  const double *tether_target; /* host FP64 [dim][n_points], finite */
} ib_structure;

/* Bytes of device workspace a context with these parameters needs. */
ib_status ib_workspace_size(const ib_grid_params *prm, int64_t n_points,
                            size_t *bytes);

/* Validate, upload the structure (the library allocates only its link,
 * layer and tether tables, plus one internal stream of default priority
 * and two events per context), precompute the line-solve factors in FP64 on
 * the host and, for step0 == 0, compute div_prev = D.u^0 and clear the
 * workspace (on `hip_stream`, a hipStream_t; NULL = default stream). */
ib_status ib_init(ib_ctx **out, const ib_grid_params *prm,
                  const ib_buffers *buf, const ib_structure *st,
                  void *hip_stream);

/* Advance `nsteps` IB-GM steps (Steps 1a-3f of Sec. "IB-GM Algorithm"):
 * interpolate u to the points, evolve X (AB2; forward Euler at n = 0),
 * link force at X^{n+1/2}, spread, explicit momentum with AB2 skew advection
 * (eq:nonlinear), one implicit sweep per axis (eq:umacstep1/2), the psi
 * sweeps (eq:PenaltyStepPart1/2) and the pressure update.  Asynchronous.
 * Within one call, Steps 1a-2b of each following step run on the context's
 * internal stream beside the previous step's psi sweeps (they need only
 * u^{n+1} and X^{n+1}); everything is joined back into `hip_stream` before
 * the call's last step, so the state seen between calls is that of plain
 * sequential steps. */
ib_status ib_step(ib_ctx *ctx, int32_t nsteps);

/* Continue from state the caller has written into the context's buffers
 * (u, nl_prev, psi, div_prev, p, X, U_prev; same addresses) as step index
 * step0 >= 0.  step0 = 0 applies the start-up rules of ib_init: it enqueues
 * div_prev = D.u^0, and the next step takes forward Euler for X and
 * N^{1/2} = N(u^0).  Asynchronous; the structure is kept.  A graph
 * captured from this context before the restart must be created again. */
ib_status ib_restart(ib_ctx *ctx, int64_t step0);

/* The caller changed u between steps (a learned correction added to the
 * velocity, a rescale, a projection): recompute div_prev = D.u from the
 * current u, the D.u^n term that the next step's pressure update (Step 3f,
 * p += psi - chi mu (D.u^{n+1} + D.u^n)/2) averages with D.u^{n+1}.  Without
 * it div_prev keeps D.u of the velocity the last step produced.  The step
 * index and the rest of the state are kept.  Asynchronous, on the context's
 * stream. */
ib_status ib_refresh_divergence(ib_ctx *ctx);

/* Wait for the stream; report the step index and IB_E_NONFINITE if any
 * position became non-finite since init, or if the velocity u or the
 * pressure p now holds a non-finite value (the message names the field; a
 * scan of the grid fields on the stream, about the cost of reading u and p
 * once). */
ib_status ib_sync(ib_ctx *ctx, int64_t *step_index);

/* Grid-field watchdog on demand: wait for the stream, scan u (every
 * component) and p, and write max |u| over all faces to *max_abs_u (host;
 * the CFL number of the step is max |u| dt / h).  IB_E_NONFINITE if u or p
 * holds a non-finite value (*max_abs_u then covers the finite values). */
ib_status ib_check_fields(ib_ctx *ctx, double *max_abs_u);

/* Step 2b on given buffers: f_out[c] (+)= sum_k F[c][k] w[k] delta_h(x - X_k)
 * for the context's grid.  X, F, w: FP64 device [dim][npts], [npts], npts at
 * most the context's n_points (in a 2-D batch, point k lives in the layer
 * the structure gave it); f_out[c]: grid dtype.  accumulate = 0 clears f_out
 * first.  Contributions are summed in LDS with atomics, so the order of
 * additions (and the last bits of the sums) varies run to run. */
ib_status ib_spread(ib_ctx *ctx, const double *X, const double *F,
                    const double *w, int64_t npts, void *const f_out[3],
                    int32_t accumulate);

/* Allocation-free spreading, for callers that cannot allocate device memory:
 * code under stream capture, tight serving loops, hosts that forbid
 * hipMalloc.  The same computation as ib_spread (the kernels are shared),
 * without a context: the grid is given by `prm` (validated as for ib_init;
 * dim, n, h and precision are used, precision choosing the grid dtype of
 * f_out; IB_FLAG_DETERMINISTIC_SPREAD in flags is honoured), and the point
 * sort and tile tables live in a fixed device array of
 * IB_SPREAD_STATIC_MAX_BYTES inside the library instead of a workspace.  That
 * array is one per GPU, reserved when the library's code is loaded on the GPU
 * and held until the process ends; its device address is looked up on the
 * first call on each device.
 *   X, F, w, npts, f_out, accumulate: as ib_spread (device pointers, FP64
 *   points [dim][npts], weights [npts], f_out[c] [n2][n1][n0] grid dtype).
 *   One problem only: 2-D needs n[2] = 1 (no batch layers).
 *   hip_stream: hipStream_t to enqueue on (NULL = default stream).
 * The tables take about (3 b + 36) npts + 12 ntiles bytes (b = 8 for
 * IB_PREC_FP64, 4 otherwise; ntiles = prod ceil(n[a] / 8)), e.g. 4 MB for
 * 65,536 points on a 256^3 FP64 grid; larger calls return IB_E_UNSUPPORTED
 * and enqueue nothing.  The call allocates nothing and clears what must
 * start at zero (the tile counts, and f_out unless accumulate) with kernels,
 * not memset nodes.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (two streams, two host threads, two captured
 * graphs in flight) race and must be serialised by the caller. */
#define IB_SPREAD_STATIC_MAX_BYTES (32u << 20)
ib_status ib_spread_static(const ib_grid_params *prm, const double *X, const double *F,
                           const double *w, int64_t npts, void *const f_out[3],
                           int32_t accumulate, void *hip_stream);

/* The Eulerian force density f of Step 2b as spread in the last step taken
 * (at X^{n+1/2}), written densely into f_out[c] (grid dtype, zero where no
 * point reached).  Enqueued on the context's stream; IB_E_STATE before the
 * first step.  ib_spread does not disturb it; the next step replaces it. */
ib_status ib_step_force(ib_ctx *ctx, void *const f_out[3]);

/* Step 1a on given buffers: U[c][k] = sum_ij u_in[c]_ij delta_h(x - X_k) h^d.
 * X, U: FP64 device [dim][npts]; u_in[c]: velocity dtype.  In a 2-D batch npts
 * must not exceed n_points and point k reads the layer the structure gave it. */
ib_status ib_interp(ib_ctx *ctx, const double *X, int64_t npts,
                    void *const u_in[3], double *U);

/* Step 2a on given buffers: F = link force of the context's structure (plus
 * its tether pulls) at positions X (FP64 device [dim][n_points] ->
 * [dim][n_points]). */
ib_status ib_force(ib_ctx *ctx, const double *X, double *F);

/* eq:TriDiagX, batched and in place: every line along `axis` (0 = x) of the
 * `nfields` arrays data + f*field_stride (elements) of shape [n2][n1][n0] is
 * replaced by the solution of the periodic system
 *     off x[i-1] + diag x[i] + off x[i+1] = rhs[i]     (indices mod n[axis]).
 * Requires |diag| > 2|off| (strict diagonal dominance, true of every matrix of
 * the method), 3 <= n[axis] <= 1024.  dtype: ib_dtype of the data; the
 * recurrence runs in FP64.  Enqueued on hip_stream. */
ib_status ib_line_solve(void *data, int32_t dtype, const int32_t n[3],
                        int32_t axis, int32_t nfields, int64_t field_stride,
                        double diag, double off, void *hip_stream);

/* Release the context's own allocations (not the caller's buffers). */
ib_status ib_destroy(ib_ctx *ctx);

/* Autotuner: time the tile shapes of the line-solve kernels (elements per
 * lane of x lines; row width and chunk length of strided lines) on this
 * context's grid, for each axis and recurrence precision, `reps` launches
 * each, on the context's own scratch fields (synchronises; call between
 * steps, not during capture), and use the fastest for the plain sweeps
 * from then on (the last momentum and psi sweeps keep the library's
 * shapes).  ib_tune_read reports the choice (0 = library default). */
ib_status ib_tune(ib_ctx *ctx, int32_t reps);
ib_status ib_tune_read(const ib_ctx *ctx, int32_t axis, int32_t fp64_recurrence,
                       int32_t *x_chunk, int32_t *s_rows, int32_t *s_chunk);

/* One hipGraph holding `steps_per_launch` IB-GM steps of each of `nctx`
 * contexts (e.g. the size classes of an ensemble of independent problems),
 * captured from the contexts' common stream `hip_stream` (a created stream:
 * the null stream cannot be captured).  Every context must be past its first
 * step (take it with ib_step), not profiling, and steps_per_launch must be a
 * multiple of each rotation period (dim).  flags: 0 = one chain of launches;
 * IB_GRAPH_BRANCHES = one independent branch per context, which the runtime
 * may run concurrently.  ib_graph_launch replays the graph `nlaunches` times
 * (asynchronous, on hip_stream) and advances every context's step index; the
 * contexts' buffers must stay where they were at capture and the contexts must
 * not be destroyed before the graph.  No memset nodes are captured. */
#define IB_GRAPH_BRANCHES 1
typedef struct ib_graph ib_graph;
ib_status ib_graph_create(ib_graph **out, ib_ctx *const *ctxs, int32_t nctx,
                          int32_t steps_per_launch, int32_t flags, void *hip_stream);
ib_status ib_graph_launch(ib_graph *graph, int32_t nlaunches);
ib_status ib_graph_destroy(ib_graph *graph);

/* Message of the last failed call on this thread ("" if none). */
const char *ib_last_error(void);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch while enabled.  ib_profile_read returns the summed duration
 * in milliseconds and the number of launches of kernel `id` (0 <=
 * id < ib_profile_count()) since the last reset, after synchronising. */
ib_status ib_profile_enable(ib_ctx *ctx, int32_t enable);
int32_t ib_profile_count(void);
const char *ib_profile_name(int32_t id);
ib_status ib_profile_read(ib_ctx *ctx, int32_t id, double *total_ms,
                          int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
