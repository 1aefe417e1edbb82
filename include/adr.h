/*
 * adr.h -- C ABI of the MI355X (gfx950) directional diffusion splitting solver.
 *
 * Method: R. Drebotiy, H. Shynkarenko, "Directional diffusion splitting method
 * for advection-diffusion-reaction model" (arXiv 2411.11041).
 *
 * Problem data follow the paper's problem statement (Sec. 2, eq. (1)-(2)):
 *   -mu Lap u + beta . grad u + sigma u = f in Omega,  u = g on Gamma,
 *   (parabolic form: u_t + ... = f, u(0) = u0),
 * mu > 0, sigma > 0 constants, beta divergence free without closed integral
 * curves in the closure of Omega.  beta and f are given as nodal values on a
 * rectangular grid covering the bounding box P = [a,b] x [c,d] of Omega
 * (eq. (20)).  All nodal arrays are row-major, index j*nx + i for the node
 * (a + i*hx, c + j*hy), hx = (b-a)/(nx-1), hy = (d-c)/(ny-1).
 *
 * The paper's boundary condition is u = 0; g (nodal Dirichlet data, read at a
 * point of Gamma through the bilinear interpolant of eq. (22)) generalises it.
 * The solver state u is a grid field with the same layout.  Its entries at
 * nodes that are not strictly inside Omega are neither read nor written: the
 * library holds g there (the curve ends take g at their boundary points, and
 * the bilinear gather near Gamma and the boundary points of the Sec. 6
 * interpolation read it).
 *
 * One sweep ("step") is eq. (10): the beta substep solves, on every beta-curve
 * (eq. (13)), the P1 line problem of eq. (16)-(17); the curve values are handed
 * to the grid by the crossing-record interpolation of Sec. 6 and read by the
 * gamma-curves (eq. (14)) through the bilinear interpolation of eq. (21)-(23);
 * the gamma substep solves eq. (18)-(19) and hands its values back to the grid.
 * The stationary problem is the limit t -> infinity (Sec. 2): sweeps with a
 * fixed pseudo time step are repeated until they stop changing u.
 *
 * Memory and threads.  Problem arrays are host memory owned by the caller and
 * copied by adr_setup.  u and every other "device" pointer are device memory
 * (e.g. a torch CUDA/HIP tensor's data_ptr) owned by the caller.  Device
 * scratch is owned by the context.  Work is queued on options.stream; calls
 * that return host values synchronise that stream.  A context must not be
 * used from two threads at once.
 *
 * Errors.  Every call returns an adr_status; nothing throws or aborts.  After a
 * failure adr_last_error(ctx) gives a message (adr_last_error(NULL) gives the
 * message of the last failed adr_setup or context-free call in this thread).
 */
#ifndef ADR_H
#define ADR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adr_ctx adr_ctx;
typedef int32_t adr_status;

enum {
    ADR_OK = 0,
    ADR_EINVAL = -1,      /* bad argument or unsupported size */
    ADR_ENOMEM = -2,      /* host or device allocation failed */
    ADR_EDEVICE = -3,     /* HIP runtime error */
    ADR_EBETA = -4,       /* |beta| vanishes or a curve does not leave Omega (closed streamline) */
    ADR_ENONFINITE = -5,  /* non-finite input or residual */
    ADR_ESINGULAR = -6,   /* a line solve met a pivot that is not finite or below options.pivot_tol
                             times its row's scale (no pivoting); u holds the last iterate */
    ADR_ENOTCONV = 1      /* warning: max_iters reached; u holds the last iterate */
};

enum { ADR_DOM_BOX = 0, ADR_DOM_DISC = 1, ADR_DOM_POLYGON = 2 };
enum { ADR_PREC_FP64 = 0, ADR_PREC_FP32_LINES = 1 };

typedef struct {
    int32_t nx, ny;            /* grid nodes over P, each >= 3 */
    double a, b, c, d;         /* P = [a,b] x [c,d] */
    int32_t domain;            /* ADR_DOM_*; BOX means Omega = P */
    int32_t n_dom_params;      /* number of doubles in dom_params */
    const double *dom_params;  /* DISC: cx, cy, r.  POLYGON: x0,y0,x1,y1,... counter-clockwise */
    double mu, sigma;          /* > 0 (sigma >= 0 accepted) */
    const double *beta1;       /* nx*ny nodal beta components (host); NULL (both) to take psi */
    const double *beta2;
    const double *f;           /* nx*ny nodal source (host) */
    const double *g;           /* nx*ny nodal Dirichlet data (host), used on and outside Gamma;
                                  NULL: zero (the paper's case) */
    const double *psi;         /* nx*ny nodal stream function (host), read only when beta1 and beta2
                                  are NULL: beta = (psi_y, -psi_x) by second-order differences
                                  (central inside, one-sided on the grid's edges) */
} adr_problem;

typedef struct {
    int32_t precision;    /* ADR_PREC_FP64: every sweep in FP64.
                             ADR_PREC_FP32_LINES: one FP64 residual sweep, then
                             fp32_sweeps FP32 increment sweeps, repeated; state,
                             residual and convergence test stay FP64 */
    int32_t fp32_sweeps;  /* FP32 sweeps per FP64 sweep in FP32_LINES mode (>= 0) */
    double theta;         /* theta of eq. (7)/(10) for the stationary sweeps, (0,1] */
    double dt;            /* pseudo time step of the stationary sweeps, > 0 */
    void *stream;         /* hipStream_t; NULL = the default stream */
    int32_t timing;       /* != 0: time each kernel with HIP events (adr_kernel_times) */
    int32_t host_only;    /* != 0: build the host geometry only, touch no device; then
                             only adr_counts, adr_export_lines, adr_export_scatter,
                             adr_export_scatter_factors, adr_export_direct and adr_destroy
                             are valid */
    int32_t graph;        /* != 0: adr_split_iterate replays its sweep blocks (m FP32 sweeps, an
                             FP64 sweep, the norm) from HIP graphs, one per block length m,
                             captured on first use on a context-owned stream ordered after
                             options.stream; the replayed launches cover every instance (a
                             finished one exits at once) where eager launches follow the lists
                             compacted to the unfinished instances; ignored when timing != 0 */
    int32_t adaptive;     /* != 0 (FP32_LINES): the number of FP32 sweeps before each FP64 sweep
                             varies from 0 to fp32_sweeps; it is chosen after each FP64 sweep so
                             that the next one falls on the sweep where the first unfinished
                             instance is expected to reach tol, from the geometric decay of its
                             measured rel (at least fp32_sweeps / 2 while several instances run) */
    int32_t split_lines;  /* line solves of a family: 0 one launch whose workgroups pick their
                             register footprint; 1 one launch per length bucket (curves of at
                             most 12, 8, 4, 2, 1 nodes per thread), each kernel with its
                             bucket's footprint and LDS, in turn on the stream; 2 the same
                             launches on three streams at once (the longest bucket on the
                             context's stream, the next and the rest on two streams of its
                             own, joined back by events; in turn inside a graph capture) */
    double pivot_tol;     /* relative pivot threshold of the line solves (ADR_ESINGULAR); <= 0:
                             64 ulp of the sweep's precision (64 * 2^-52 FP64, 64 * 2^-23 FP32) */
    int32_t splitting;    /* time steps of adr_time_step's paper scheme: 0 the order of eq. (10)
                             (beta substep, then gamma substep); 1 symmetric: beta over dt/2,
                             gamma over dt, beta over dt/2 */
    int32_t stabilize;    /* beta-lines: 0 plain Galerkin (eq. (17)); 1 exponentially fitted
                             (the paper's further work on singularly perturbed lines): element
                             e's stiffness scaled by Pe coth(Pe), Pe = |beta|_e h_e / (2 mu),
                             |beta|_e the mean of its nodal values; nodally exact for
                             -mu u'' + |beta| u' = 0 with constant |beta| on a uniform line */
    int32_t krylov;       /* stationary solve: 0 the sweeps of eq. (10) (fixed-point iteration);
                             m in 1..200: GMRES(m) on (I - T) U = c, the same fixed point (T the
                             linear part of a sweep, c = Phi(0)), FP64 in either precision: each
                             application of I - T is one FP64 sweep, each restart recomputes the
                             exact residual Phi(U) - U (one FP64 sweep) and stops at
                             rel = |Phi(U) - U| / |Phi(0)| <= tol; iters counts the sweeps; the
                             iterate returned is that U (not Phi(U)).  Not for the judged solve */
    int32_t transfer;     /* how values pass between the families: 0 through the grid (Sec. 6:
                             the scatter and the bilinear gather of eq. (22)); 1 directly at
                             the intersections of the two families' segments (the
                             conclusions' interpolation-free transfer: a node of a curve takes
                             the linear interpolant, in arc length along its curve, of the
                             other family's P1 values at the nearest intersections before and
                             after it, its curve's Dirichlet end where a side has none).  With
                             1, adr_split_iterate iterates on the gamma-curve values, every
                             sweep FP64 (any precision; graph ignored; krylov must be 0; no
                             fallback start): start = the bilinear gather of u onto the
                             gamma-curves, rel = |v' - v|_2 / |Phi(0)|_2 over the interior
                             gamma-curve nodes, u out = the scatter of Sec. 6 of the last
                             gamma values.  The other calls keep the grid transfer */
    int32_t increments;   /* FP32_LINES mode with transfer = 0: 0 the FP32 increment sweeps use
                             the grid transfer, the linear part of the FP64 sweeps themselves; 1
                             they use the direct transfer of `transfer` (the same linear map
                             up to the difference of the two transfers, an approximation that
                             is cheaper: two line kernels per sweep and no scatter): each
                             block gathers the FP64 sweep's update onto the gamma-curves, runs
                             its FP32 sweeps on the curve values, and adds their sum to the
                             state by one scatter.  The FP64 sweeps, and with them the
                             iterate's fixed point, the residual and the stop, are the grid
                             route's in either case; only the sweep count may differ.  Set-up
                             builds the direct-transfer records (adr_autotune then also times
                             both kinds of increment sweeps).  No effect with transfer = 1,
                             whose increments are direct already; another value: ADR_EINVAL */
} adr_options;

/* Builds the curve families of every instance (host, FP64) and uploads the
 * line and transfer tables.  probs: n_probs instances solved together (one
 * launch per kernel covers all of them).  On success *out is a new context;
 * on failure *out = NULL.  Errors: ADR_EINVAL (sizes, mu <= 0, theta or dt out
 * of range, a line longer than the solver's LDS capacity), ADR_EBETA (|beta| =
 * 0 on a curve, a curve longer than four perimeters), ADR_ENONFINITE (NaN/Inf
 * input), ADR_ENOMEM, ADR_EDEVICE. */
adr_status adr_setup(const adr_problem *probs, int32_t n_probs, const adr_options *opt,
                     adr_ctx **out);

/* Packed layout of u over the instances: instance i occupies
 * offsets[i] .. offsets[i+1]-1 (offsets has n_probs+1 entries, host), row-major
 * (node (x, y) at offsets[i] + y nx + x).  The calls below read and write the
 * interior nodes of u only (nodes strictly inside the domain); the others are
 * the zero Dirichlet data: they are read as 0 and left unchanged.  Inside a
 * call the library keeps its own copy of the state in a blocked layout. */
adr_status adr_layout(const adr_ctx *ctx, int64_t *offsets);

/* Counts (host out, each may be NULL): interior grid nodes, beta-lines,
 * gamma-lines, interior (unknown) beta-line nodes and gamma-line nodes, summed
 * over instances. */
adr_status adr_counts(const adr_ctx *ctx, int64_t *grid_unknowns, int64_t *lines_b,
                      int64_t *lines_g, int64_t *line_unknowns_b, int64_t *line_unknowns_g);

/* New coefficients and sources on the same curves: probs (n_probs = the
 * set-up's count) must have the set-up's grids and domains; beta is not read
 * (the traced curves are kept); mu, sigma and f replace the old ones.  The
 * loads of eq. (17) and |Phi(0)| are recomputed.  Errors: ADR_EINVAL (count,
 * grid or domain mismatch, mu <= 0), ADR_ENONFINITE (f).  Synchronises. */
adr_status adr_update(adr_ctx *ctx, const adr_problem *probs, int32_t n_probs);

/* Stationary solve (Sec. 2 limit, eq. (10) sweeps).  u: device FP64, packed
 * layout; in: initial iterate, out: last iterate.  Each sweep k maps U_k to
 * U_{k+1} = Phi(U_k); an instance stops at the first FP64 sweep with
 *   rel = |U_{k+1} - U_k|_2 / |Phi(0)|_2 <= tol      (interior nodes).
 * Sweep order: one FP64 sweep, then blocks of (fp32_sweeps FP32 sweeps, one
 * FP64 sweep) in FP32_LINES mode (whole blocks only: at most max_iters
 * sweeps; the block length varies with options.adaptive); every sweep is FP64
 * in FP64 mode; rel is measured on the FP64 sweeps only.  iters (host, n_probs, may be NULL): sweeps
 * applied per instance; rel_res (host, n_probs, may be NULL): last measured
 * rel.  Returns ADR_ENOTCONV if an instance hit max_iters, ADR_ENONFINITE if a
 * residual is not finite. */
adr_status adr_split_iterate(adr_ctx *ctx, double *u, int32_t max_iters, double tol,
                             int32_t *iters, double *rel_res);

/* adr_split_iterate from the start u, judged by the method's own residual
 * against a fallback start (a predicted start judged against the eq. (11)
 * iterate, say).  The FP64 residual of fallback (as adr_residual) is computed
 * first.  The first sweep from u then yields u's residual.  Every instance
 * whose residual is not below the fallback's, or is not finite, restarts from
 * its fallback values.  The restart costs one more FP64 sweep, which the other
 * unfinished instances take as a sweep of their own.  Each instance then
 * iterates as in adr_split_iterate to the same fixed point.
 *   fallback: device FP64, packed layout (read only).
 *   used_fallback: host, n_probs (may be NULL); 1 where the instance restarted.
 *   iters: counts every sweep, the restart's included.
 * Otherwise as adr_split_iterate; max_iters >= 1.  Synchronises once more
 * than adr_split_iterate (after the first sweep). */
adr_status adr_split_iterate_judged(adr_ctx *ctx, double *u, const double *fallback, int32_t max_iters,
                                    double tol, int32_t *iters, double *rel_res, int32_t *used_fallback);

/* Autotuner of the batched stationary solve (FP32_LINES precision only).  Each
 * trial runs the stationary solve from zero twice on `work` (device FP64,
 * packed layout, overwritten) and times the second run on the host clock (the
 * first also captures the graph in graph mode).  It tunes in three steps:
 *   1. the line launches (options.split_lines 0, 1 and 2), under the context's
 *      current schedule;
 *   2. with the faster of those, each candidate schedule: a fixed count of
 *      FP32 sweeps per FP64 sweep (2, 3, 4, 6) and the adaptive schedule
 *      with at most 6, 8, 12, 16 or 24; each with both kinds of increment
 *      sweeps (options.increments) when the context has the direct-transfer
 *      records (set up with increments = 1);
 *   3. GMRES(m) (options.krylov) with m = 10, 20, 30, kept if faster than the
 *      best schedule (grid transfer only).
 * With bucketed launches, between steps 1 and 2, each length bucket's
 * workgroup shape (adr_set_line_shapes) is chosen from its FP32 line solves
 * timed alone.  A context with the direct transfer (options.transfer = 1) is
 * tuned the same way on its own sweeps and line solves, without step 3.  The fastest choices stay in the context.  Outputs (host, each
 * may be NULL): best_fp32_sweeps and best_adaptive (the count or maximum, and
 * the adaptive flag), best_ms (its time), best_split (the launch choice),
 * best_shapes (5 entries, the shape of each bucket), best_krylov (0, or the
 * GMRES restart length chosen), best_increments (options.increments chosen).
 * Kernel timers (timing
 * mode) are reset afterwards.  Synchronises. */
adr_status adr_autotune(adr_ctx *ctx, double *work, int32_t max_iters, double tol, int32_t *best_fp32_sweeps,
                        int32_t *best_adaptive, double *best_ms, int32_t *best_split, int32_t *best_shapes,
                        int32_t *best_krylov, int32_t *best_increments);

/* Graph replay of the stationary solve's blocks on (1) or off (0) from now on
 * (options.graph); captured graphs are dropped.  Errors: ADR_EINVAL (host-only
 * context). */
adr_status adr_set_graph(adr_ctx *ctx, int32_t on);

/* Workgroup shapes of the bucketed line launches (options.split_lines != 0):
 * shapes[b] for bucket b = 0..4 (curves of at most 3072, 2048, 1024, 512, 256
 * nodes) selects rows per thread x threads per curve:
 *   bucket 0: 0 = 12 x 256, 1 = 6 x 512
 *   bucket 1: 0 = 8 x 256,  1 = 4 x 512
 *   bucket 2: 0 = 4 x 256, 1 = 8 x 128, 2 = 2 x 512
 *   bucket 3: 0 = 4 x 128, 1 = 2 x 256, 2 = 8 x 64
 *   bucket 4: 0 = 4 x 64,  1 = 2 x 128, 2 = 1 x 256
 * Every shape solves the same systems (the partition of a curve's rows among
 * the threads, and so the rounding, differs).  shapes: host, 5 entries.  Set-up
 * gives 0 everywhere.  Errors: ADR_EINVAL (a shape out of range). */
adr_status adr_set_line_shapes(adr_ctx *ctx, const int32_t *shapes);

/* Parabolic march (eq. (2) discretised in time by eq. (7), split by eq. (10)).
 * u: device FP64 packed, in: u_n, out: u_{n+nsteps}; dt > 0; source f and
 * Dirichlet data g included.
 *   inner_max = 0 (the paper's scheme): one splitting step of eq. (10) per time
 *     step with the given theta in (0,1], FP64 (options.splitting = 1: the
 *     symmetric step beta dt/2, gamma dt, beta dt/2).  Asynchronous.
 *   inner_max > 0 (splitting iterated per step): implicit Euler, theta = 1;
 *     each step (u - u_n)/dt + A u = f is solved as the stationary problem
 *     with reaction sigma + 1/dt and the beta-curves' load L + M (G u_n)/dt
 *     (G the bilinear gather of eq. (22), M the P1 mass rows), by the
 *     stationary iteration of adr_split_iterate from u_n (the context's pseudo
 *     step, precision, schedule and launches) to rel <= inner_tol, at most
 *     inner_max sweeps.  inner_iters (host, nsteps * n_probs, may be NULL):
 *     sweeps of step s for instance i at [s * n_probs + i].  Returns
 *     ADR_ENOTCONV if some step hit inner_max (the march goes on), and stops
 *     at the first error (ADR_ESINGULAR, ADR_ENONFINITE).  Synchronises.
 *     The context's stationary coefficients are unchanged afterwards.
 * Errors: ADR_EINVAL (arguments; theta != 1 with inner_max > 0). */
adr_status adr_time_step(adr_ctx *ctx, double *u, double theta, double dt, int32_t nsteps, int32_t inner_max,
                         double inner_tol, int32_t *inner_iters);

/* rel_res[i] = |Phi(U) - U|_2 / |Phi(0)|_2 of the stationary sweep for the given
 * u (device FP64, unchanged), in FP64.  rel_res: host, n_probs.  Returns
 * ADR_ENONFINITE when some entry is not finite; rel_res is written for every
 * instance all the same. */
adr_status adr_residual(adr_ctx *ctx, const double *u, double *rel_res);

/* Initial iterate of eq. (11): s(u0, v) = <l, v> solved on every beta-curve,
 * handed to the grid.  u: device FP64 packed (written).  Asynchronous. */
adr_status adr_initial_guess(adr_ctx *ctx, double *u);

/* Geometry export for testing: line node coordinates of one instance and
 * family (0 = beta-curves, 1 = gamma-curves).  Call with NULL arrays to get
 * *n_lines and *n_nodes, then with offsets (n_lines+1), x, y (n_nodes) host
 * buffers. */
adr_status adr_export_lines(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_lines,
                            int64_t *n_nodes, int64_t *offsets, double *x, double *y);

/* Test export (host-only contexts): the scatter stencil of Sec. 6 that the
 * set-up built for one instance and family, one row per interior grid node in
 * row-major order.  Row r is grid node node[r] (row-major index in the
 * instance's grid); its value is sum over the 4 slots s (horizontal low,
 * horizontal high, vertical low, vertical high) of ca[4r+s] v[k] + cb[4r+s]
 * v[k+1], k = k[4r+s] a node index of the family local to the instance
 * (offsets of adr_export_lines); k = -1 marks a boundary point of Gamma
 * (weights 0); gb[r] is the Dirichlet data the row's boundary points carry
 * (their interpolation weights times g there), added to the row's value in
 * the sweeps of the state.  Call with NULL arrays to get *n_rows, then with
 * node, gb (n_rows) and k, ca, cb (4 n_rows) host buffers (each may be NULL).
 * Errors: ADR_EINVAL (a device context, an index out of range). */
adr_status adr_export_scatter(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_rows,
                              int32_t *node, int32_t *k, double *ca, double *cb, double *gb);

/* Test export (host-only contexts): the same stencil in the factored form the
 * FP32 sweeps read (quantised on upload: wh exactly, lam to 15 and t to 16
 * bits).  Row r's value is wh (lam_h a_0 + (1 - lam_h) a_1) + (1 - wh)
 * (lam_v a_2 + (1 - lam_v) a_3) with a_s = (1 - t_s) v[k] + t_s v[k+1] the
 * P1 value of slot s's record (k from adr_export_scatter; zero Dirichlet data
 * where k = -1).  wh (n_rows) in {0, 1/2, 1}; lam (2 n_rows: horizontal,
 * vertical); t (4 n_rows).  Errors: ADR_EINVAL (a device context, an index
 * out of range). */
adr_status adr_export_scatter_factors(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_rows,
                                      double *wh, double *lam, double *t);

/* Test export (host-only contexts set up with options.transfer = 1 or
 * options.increments = 1): the direct-transfer records onto every node of one instance's family (0 beta,
 * 1 gamma) from the other family's line values, in the node order of
 * adr_export_lines.  Node q's value is
 *   (k[2q] >= 0 ? w[4q] v[k[2q]] + w[4q+1] v[k[2q]+1] : w[4q] x_first)
 * + (k[2q+1] >= 0 ? w[4q+2] v[k[2q+1]] + w[4q+3] v[k[2q+1]+1] : w[4q+2] x_last)
 * with v the other family's values (node indices local to the instance) and
 * x_first, x_last the Dirichlet values at the ends of q's own curve; end nodes
 * carry k = -1 and zero weights.  Call with NULL arrays to get *n_nodes, then
 * with k (2 n_nodes) and w (4 n_nodes) host buffers.  Errors: ADR_EINVAL (a
 * device context, a context without the records, an index out of range). */
adr_status adr_export_direct(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_nodes, int32_t *k,
                             double *w);

/* Test export (host-only contexts with the direct-transfer records): the
 * records of adr_export_direct as the FP32 increment sweeps receive them, 10
 * bytes per node (source nodes local to the instance):
 *   k0[q]  the left bracket's source node, or the right one's when kd[q] =
 *          -32766 (no left bracket: the curve's first end), or -1;
 *   kd[q]  the right bracket's source node minus k0[q], or -32767 (no right
 *          bracket: the curve's last end), or -32768 (farther than 32765 from
 *          k0: the device reads the full record);
 *   wp[q]  bits 0-9: the left bracket's weight wL as a multiple of 1/1023;
 *          bits 10-20 and 21-31: the positions tL, tR on the two source
 *          segments as multiples of 1/2047.
 * Node q's weights are then wL(1 - tL), wL tL, wR(1 - tR), wR tR with
 * wR = 1 - wL (each within 2^-11 of the FP64 record's, sum 1).  Call with NULL
 * arrays to get *n_nodes.  Errors: ADR_EINVAL (a device context, a context
 * without the records, an index out of range). */
adr_status adr_export_direct_packed(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_nodes,
                                    int32_t *k0, int16_t *kd, uint32_t *wp);

/* Per-launch HIP-event timing on (1) or off (0) from now on (the set-up
 * option's initial value).  Each timed launch records two events on the
 * context's stream, which adds a few microseconds between launches.  Pending
 * records are folded into the totals of adr_kernel_times first.  Errors:
 * ADR_EINVAL (host-only context). */
adr_status adr_set_timing(adr_ctx *ctx, int32_t on);

/* Kernel timing (options.timing != 0): for kernel class k (0 beta-line solve,
 * 1 gamma-line solve, 2 beta scatter, 3 gamma scatter/update, 4 norm), total
 * milliseconds, launch count and work of kernels of the given precision (0
 * FP64, 1 FP32) since setup or the last reset of that precision.  Work is the
 * sum over the timed launches of what each one covered: line unknowns of the
 * curves in its list (classes 0, 1) or interior grid nodes of its scatter
 * blocks (classes 2, 3), over the lists compacted to the unfinished instances
 * when a batched solve compacts them, else over all instances; 0 for the norm.
 * With direct increments (options.increments = 1) the FP32 classes 2 and 3
 * time each block's gather of the update onto the gamma-curves (work: gamma
 * line unknowns) and its closing scatter.
 * ms_out, count_out and work_out hold 5 entries (each may be NULL).  reset !=
 * 0 clears that precision's counters after reading.  Synchronises the stream. */
adr_status adr_kernel_times(adr_ctx *ctx, int32_t precision, double *ms_out, int64_t *count_out,
                            int64_t *work_out, int32_t reset);

/* Measurement export (not part of the method): dst = src, `bytes` bytes of
 * device memory (a multiple of 16; both pointers 16-byte aligned), a plain
 * copy kernel queued on `stream` (hipStream_t, NULL = default): the measured
 * HBM bandwidth against which the kernels' rooflines are also quoted.
 * Errors: ADR_EINVAL (size or alignment), ADR_EDEVICE.  Asynchronous. */
adr_status adr_copy_probe(const void *src, void *dst, int64_t bytes, void *stream);

/* Batched tridiagonal solve on given rows: the line systems of eq. (16)-(19)
 * (P1 elements on a curve, Dirichlet ends eliminated) with coefficients the
 * caller supplies, solved by the partitioned scheme of the line solver (no
 * pivoting), for systems of any length.  A test and building-block export;
 * context free.
 *   n_lines systems; system l has rows off[l] .. off[l+1]-1 (off: device
 *   int64, n_lines + 1 entries, non-decreasing); n_rows = off[n_lines] -
 *   off[0] (host; a smaller value leaves x unwritten).
 *   Row r: lo[r] x[r-1] + di[r] x[r] + up[r] x[r+1] = rhs[r]; lo of a
 *   system's first row and up of its last are ignored.  lo, di, up, rhs:
 *   device FP64 (read only); x: device FP64 (written; may not alias them).
 *   singular: device int32, n_lines (may be NULL): 1 where a pivot was not
 *   finite or below pivot_tol times its row's scale (|di| + |l c'|); x is
 *   then unreliable for that system.  pivot_tol <= 0: 64 * 2^-52.
 *   Systems are cut into chunks of 32 rows; the chunks' reduced rows and the
 *   separators' values (about 88 B per chunk + 8 B per system) live in device
 *   scratch from the stream-ordered allocator (hipMallocAsync / hipFreeAsync
 *   on `stream`).
 * Asynchronous on stream (hipStream_t, NULL = default).  Errors: ADR_EINVAL
 * (sizes, null arrays), ADR_ENOMEM, ADR_EDEVICE; messages through
 * adr_last_error(NULL). */
adr_status adr_line_solve(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo, const double *di,
                          const double *up, const double *rhs, double *x, int32_t *singular, double pivot_tol,
                          void *stream);

/* adr_line_solve for callers that cannot allocate (work captured into a HIP
 * graph, serving loops, harnesses that forbid hipMalloc): the same kernels and
 * results, with the scratch in a fixed device array of the library instead of
 * the stream-ordered allocator.  The array holds 16 MiB per device (the first
 * call on a device looks its address up; the array stays until the process
 * ends), enough for about 6 million rows; a request above it (about 88 B per
 * 32 rows plus 8 B per system) is refused with ADR_EINVAL before anything is
 * queued.  Calls no allocating routine.  Every call on one device shares that
 * device's array: calls whose work overlaps on one device (other streams,
 * other threads) race and must be ordered by the caller.  Nothing in the
 * array needs to start at zero.  Arguments, results and other errors as
 * adr_line_solve. */
adr_status adr_line_solve_noalloc(int64_t n_lines, int64_t n_rows, const int64_t *off, const double *lo,
                                  const double *di, const double *up, const double *rhs, double *x,
                                  int32_t *singular, double pivot_tol, void *stream);

adr_status adr_destroy(adr_ctx *ctx);
const char *adr_last_error(const adr_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADR_H */
