/*
 * rkl.h -- C ABI of librkl: RKL2 super-time-stepping of field-aligned
 * (anisotropic) thermal conduction on one AMD Instinct MI355X (gfx950).
 *
 * Method: Vaidya, Prasad, Mignone, Sharma & Rickler (2017), "Scalable
 * explicit implementation of anisotropic diffusion with Runge-Kutta-Legendre
 * super-time-stepping", arXiv:1702.05487.
 *
 * The library evolves a cell-centred temperature T under the operator-split
 * conduction equation d(rho eps)/dt = -div F_c (Sec. 3, Eq. scalar_diffusion)
 * with rho eps = rho T/(gamma-1), i.e. dT/dt = (gamma-1)/rho (-div F_c),
 * on Cartesian grids whose axes are periodic or outflow.  F_c is the
 * harmonic blend of the classical field-aligned flux -kappa_par b (b.grad T)
 * (plus an optional -kappa_perp (grad T - b (b.grad T)) term) and the
 * saturated flux q = 5 phi rho c_iso^3 (Sec. 2, Eqs. Fc, Fclass, Fsat; q at
 * the face temperature or, upwinded as Sec. 3 says, at the temperature of the
 * cell the heat leaves), discretised with
 * the conservative second-order face differences of Sec. 3 and, optionally,
 * monotonized-central limited transverse gradients (Sec. 3.4, Appendix B).
 * A super-step of length dt_hyp takes s RKL2 stages (Appendix A, Eq.
 * rkl2scheme), s from Eq. RKL-s rounded as 1 + floor(s) (Sec. 4.1), with the
 * explicit step dt_par of Eq. dt_exp.
 *
 * Conventions common to every entry point:
 *   - Fields are device pointers, C order [n2][n1][n0] (axis 0 fastest).
 *     T is double.  b (the unit vector b = B/|B|, one per cell) is three such
 *     arrays back to back (component-major, 3*N elements); it is double for
 *     RKL_FP64 plans and float for RKL_MIXED plans.  b is not checked: its
 *     length and finiteness are the caller's (a NaN in b gives a face flux
 *     of zero under saturation and NaN without it, and the RKL_FLAG_*
 *     bits, which describe T, do not report it).
 *   - The caller owns every pointer it passes; the plan owns its scratch.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; entry points that must read a device result back say
 *     so and synchronise that stream.
 *   - Every entry point returns an rkl_status; nothing aborts and no C++
 *     exception crosses the ABI.  rkl_last_error() gives a message for the
 *     calling thread's last non-OK status.
 *   - One plan must not be used from two streams or threads at once.
 */
#ifndef RKL_H
#define RKL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rkl_plan_s *rkl_plan_t;

typedef enum {
    RKL_OK = 0,
    RKL_EINVAL = 1,     /* invalid argument or descriptor */
    RKL_ENOMEM = 2,     /* device allocation failed */
    RKL_EDEVICE = 3,    /* HIP runtime error (launch, copy, sync) */
    RKL_ESTAGES = 4,    /* stage count above the plan's smax; T left unchanged */
    RKL_ESTATE = 5      /* call out of order (e.g. launch before capture) */
} rkl_status;

enum { RKL_FP64 = 0, RKL_MIXED = 1 };   /* flux arithmetic: FP64, or FP32 with FP64 stage recurrence */
enum { RKL_RKL2 = 0, RKL_RKL1 = 1 };    /* super-step scheme: second- or first-order Legendre (Sec. 3.3) */
enum { RKL_LIM_NONE = 0, RKL_LIM_MC = 1 };
/* saturated flux: off; q at the face temperature (central); q at the
 * temperature of the upwind cell, the one the classical face flux leaves
 * (the upwind treatment of the saturated term that Sec. 3 names) */
enum { RKL_SAT_NONE = 0, RKL_SAT_CENTRAL = 1, RKL_SAT_UPWIND = 2 };
/* per-axis boundary: periodic; outflow (the cells beyond an edge repeat
 * the edge cell's T and b at every stage: zero-gradient ghost cells); or
 * fixed (Dirichlet: the temperatures beyond the edges are given by the
 * caller, see rkl_set_ghosts, and b repeats the edge cell's), the
 * non-periodic edges of the paper's tests (Sec. 4.1.1 takes the Gaussian
 * test's edge values from the exact solution). */
enum { RKL_BC_PERIODIC = 0, RKL_BC_OUTFLOW = 1, RKL_BC_FIXED = 2 };

/* flag bits reported by rkl_query.  RKL_FLAG_NONPOS reports the negative
 * temperatures the paper warns about: unlimited transverse gradients can
 * drive T below zero near large gradients (Sec. 4.1.3, and the local
 * thermal instability runs of Sec. 4.2.2, which blow up without limiters),
 * and the paper recommends the limiter once T falls below a floor.  The
 * library applies no floor; the flag lets the caller switch to the MC
 * limiter or floor T. */
enum {
    RKL_FLAG_NONPOS = 1u,     /* some input temperature <= 0 (conductivity clipped at 0) */
    RKL_FLAG_NONFINITE = 2u,  /* some input temperature is NaN or infinite */
    RKL_FLAG_STAGES = 4u,     /* the stage count exceeded smax; that grid was not advanced */
    RKL_FLAG_ABORTED = 8u     /* the last persistent batched launch gave up a wait (results invalid) */
};

/* One grid and its conduction parameters. */
typedef struct {
    int32_t ndim;         /* 1, 2 or 3; n[d] must be 1 for d >= ndim */
    int32_t n[3];         /* cells along axes 0, 1, 2 (axis 0 fastest in memory) */
    double h[3];          /* cell widths, > 0 */
    int32_t limiter;      /* RKL_LIM_NONE: transverse gradient = mean of the four
                             one-sided differences; RKL_LIM_MC: MC(MC(a1,a2), MC(a3,a4)) */
    int32_t saturation;   /* RKL_SAT_NONE: classical flux; RKL_SAT_CENTRAL or
                             RKL_SAT_UPWIND: blend q/(q+|F|) F (Eq. Fc) */
    double phi;           /* saturation factor of Eq. Fsat (0.3 in the paper) */
    double kappa0;        /* kappa_par = kappa0 * max(T,0)^kappa_exp, kappa0 >= 0 */
    double kappa_exp;     /* >= 0 (2.5 for Spitzer conduction) */
    double kperp_ratio;   /* kappa_perp = kperp_ratio * kappa_par, in [0, 1] */
    double rho;           /* frozen density, > 0 */
    double gamma;         /* ratio of specific heats, > 1 */
    double cp;            /* parabolic Courant number of Eq. dt_exp, in (0, 1/2] */
    int32_t boundary[3];  /* per axis: RKL_BC_PERIODIC (0, the default of a
                             zeroed descriptor), RKL_BC_OUTFLOW or, for
                             d < ndim, RKL_BC_FIXED */
} rkl_grid_desc;

typedef struct {
    int32_t precision;    /* RKL_FP64 or RKL_MIXED */
    int32_t variant;      /* stencil kernel variant (see rkl_variant_info); -1 = library default */
    int32_t smax;         /* largest stage count accepted (coefficient table size); 0 = 1024
                             for one grid, 64 for several (a batched super-step issues
                             one stage launch per stage up to smax) */
    int32_t scheme;       /* RKL_RKL2 (default) or RKL_RKL1; the batched entry points
                             implement RKL2 only */
} rkl_options;

/*
 * rkl_plan: validate `ngrids` grid descriptors and allocate the plan's device
 * scratch (two FP64 stage buffers -- four if opt->variant is a two-stage
 * variant --, the tau*M(Y0) buffer, reduction space and the RKL2 coefficient
 * table for s = 2..smax, Appendix A).  Grids are packed back to back for the
 * batched entry points; rkl_grid_offset gives each grid's first cell.  The
 * device current at this call is the plan's device: every later call on the
 * plan (except rkl_destroy, which switches to it) returns RKL_EINVAL while
 * another device is current.  opt may be NULL (RKL_FP64, default variant,
 * default smax).  Synchronises the device before returning, so the plan is
 * ready for launches on any stream.
 * Errors: RKL_EINVAL for a bad descriptor or option (including a two-stage
 * variant for a plan that cannot use it), RKL_ENOMEM, RKL_EDEVICE.
 */
rkl_status rkl_plan(const rkl_grid_desc *grids, int32_t ngrids, const rkl_options *opt,
                    rkl_plan_t *plan_out);

/* rkl_destroy: free the plan and its graph (NULL is accepted).  Synchronises
 * the plan's device; the caller's current device is kept. */
rkl_status rkl_destroy(rkl_plan_t plan);

/* Cells in the packed layout before grid `grid` (b of that grid starts at
 * 3 * offset).  Returns -1 for a bad plan or index. */
int64_t rkl_grid_offset(rkl_plan_t plan, int32_t grid);

/*
 * rkl_set_ghosts: the ghost temperatures of a fixed (Dirichlet) axis of one
 * grid, beyond its low edge (lo) and its high edge (hi) -- the paper's
 * Gaussian test (Sec. 4.1.1) takes these from the exact solution.  Each is
 * a device array of (n_b + 2) x (n_a + 2) doubles, a < b the grid's other
 * two axes: the value for transverse position (j_a, j_b), j in [-1, n], at
 * index (j_b + 1) * (n_a + 2) + (j_a + 1).  A position beyond the edges of
 * several fixed axes takes the layer of the lowest of them; a transverse
 * index is wrapped on a periodic axis, clamped to [0, n-1] on an outflow
 * axis and to [-1, n] on a fixed one; positions further beyond an edge take
 * that edge's layer.  The values hold for every stage of a super-step (for
 * second order in time with time-dependent edge values, give them at the
 * super-step's midpoint).  The plan keeps the pointers, not the values: the
 * caller owns the arrays, keeps them alive while the plan may use them and
 * may rewrite them between calls (stream order).  Used by rkl_superstep (both
 * schemes), rkl_superstep_async, rkl_flux_div, rkl_subcycle and rkl_aag,
 * which return RKL_EINVAL while a fixed axis has no layers; the batched entry
 * points and rkl_superstep_noalloc do not take fixed axes (RKL_EINVAL), and
 * neither do the fused variants (periodic grids only).  dt_par (Eq. dt_exp)
 * is taken over the grid's own cells.
 * Errors: RKL_EINVAL (bad plan, grid or axis, an axis that is not fixed, a
 * NULL pointer).
 */
rkl_status rkl_set_ghosts(rkl_plan_t plan, int32_t grid, int32_t axis, const double *lo, const double *hi);

/*
 * rkl_flux_div: out[i] = (gamma-1)/rho * ( -div F_c(T) )_i for one grid
 * (Sec. 3: the face-difference divergence of the flux of Eqs. Fc-Fsat), in
 * the plan's flux precision, written as double.  T, b, out: device pointers
 * of that grid's size; out must not alias T or b (RKL_EINVAL).  No host
 * synchronisation.
 */
rkl_status rkl_flux_div(rkl_plan_t plan, int32_t grid, const double *T, const void *b,
                        double *out, void *stream);

/*
 * rkl_dt_par: the explicit parabolic step of Eq. dt_exp with the HD
 * diffusivity, dt_par = cp / max_i[(gamma-1)/rho * kappa_par(T_i) * sum_d h_d^-2]
 * (+inf when the maximum is 0).  Writes the host double *dt_par_out and
 * synchronises `stream`.
 */
rkl_status rkl_dt_par(rkl_plan_t plan, int32_t grid, const double *T, double *dt_par_out,
                      void *stream);

/*
 * rkl_superstep: one RKL2 super-step of length dt_hyp on one grid, T updated
 * in place (Appendix A, Eq. rkl2scheme: Y0 = T, Y1 = Y0 + mut_1 tau M(Y0),
 * Y_j = mu_j Y_{j-1} + nu_j Y_{j-2} + (1-mu_j-nu_j) Y0 + mut_j tau M(Y_{j-1})
 * + gt_j tau M(Y0), T = Y_s), where M is the flux-divergence operator above
 * evaluated on each stage's own temperature.  s = 1 + floor(root of
 * dt_hyp/dt_par = (s^2+s-2)/4) is computed on the device (Eq. RKL-s); this
 * entry point reads it back once (one synchronisation of `stream`) to size
 * the launch sequence, and stores it in *s_out (host pointer, may be NULL).
 * RKL_ESTAGES (T unchanged) if s > smax.  b must not alias T (RKL_EINVAL;
 * likewise for the other entry points that take T and b).
 * With scheme RKL_RKL1 the super-step is the first-order scheme: stability
 * polynomial P_s(1 + w1 tau lambda), w1 = 2/(s^2+s), stages Y_1 = Y_0 +
 * w1 tau M(Y_0), Y_j = (2j-1)/j (Y_{j-1} + w1 tau M(Y_{j-1})) - (j-1)/j Y_{j-2},
 * and s from dt_hyp = dt_par (s^2+s)/2 rounded as for RKL2 (s >= 1; s = 1 is
 * one forward-Euler step).
 * For a super-step with no host synchronisation (HIP graph capture), use
 * rkl_superstep_async; it gives the same bits as this entry point.
 */
rkl_status rkl_superstep(rkl_plan_t plan, int32_t grid, double *T, const void *b,
                         double dt_hyp, int32_t *s_out, void *stream);

/*
 * rkl_superstep_async: the RKL2 super-step of rkl_superstep (Appendix A, Eq.
 * rkl2scheme; s from Eq. RKL-s) with no host synchronisation and no
 * allocation, so it can be captured in a HIP graph.  s is computed on the
 * device and never read back: the call enqueues one reduction, one finalize
 * launch and s_cap stage launches; stage j does nothing when j > s.  If
 * s > s_cap, every stage does nothing (T unchanged) and the grid is flagged
 * RKL_FLAG_STAGES (rkl_query).  s_out: device int32 (may be NULL) receiving
 * s.  s_cap in [2, the plan's smax] (RKL_EINVAL otherwise); RKL2 plans only
 * (RKL_EINVAL for RKL1).  Uses the plan's one-stage stencil variant (variant
 * 0 while a two-stage variant is selected); the same bits as rkl_superstep
 * for the same variant.  An empty stage launch costs a few microseconds, so
 * s_cap should be near the largest s expected.
 */
rkl_status rkl_superstep_async(rkl_plan_t plan, int32_t grid, double *T, const void *b, double dt_hyp,
                               int32_t s_cap, int32_t *s_out, void *stream);

/*
 * rkl_supersteps_async: nsteps super-steps of rkl_superstep_async (Appendix A,
 * Eq. rkl2scheme; s from Eq. RKL-s) one after another on the same T, b and
 * dt_hyp, enqueued with no host synchronisation and no allocation.  Each
 * super-step needs the extrema of its starting T for dt_par and the FP32
 * reference temperature (Sec. 3.1, Eq. dt_exp).  On 3-D grids without fixed
 * axes the last stage of each super-step keeps the extrema of the T it
 * writes, so every super-step after the first skips the reduction pass over
 * T (a read of the whole field); other grids take the pass each time.  The
 * extrema are the same numbers either way, so the results have the same
 * bits as nsteps calls of rkl_superstep_async.  s_out: device int32 array
 * of nsteps entries (may be NULL) receiving each super-step's s; a
 * super-step with s > s_cap leaves T unchanged and is flagged
 * RKL_FLAG_STAGES (rkl_query), and the next one takes the reduction pass.
 * nsteps >= 1 and s_cap in [2, the plan's smax] (RKL_EINVAL otherwise);
 * RKL2 plans only.  T must not change outside these launches while they
 * run.
 */
rkl_status rkl_supersteps_async(rkl_plan_t plan, int32_t grid, double *T, const void *b, double dt_hyp,
                                int32_t nsteps, int32_t s_cap, int32_t *s_out, void *stream);

/*
 * rkl_superstep_noalloc: for callers that cannot allocate device memory --
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The super-step of rkl_superstep_async (RKL2, s on the device,
 * s_cap stage launches, no host synchronisation) on one grid described by
 * *grid, with no plan and no allocation of any kind: its scratch is a static
 * device array inside the library, 8 B x 3 x RKL_NOALLOC_MAX_CELLS plus a
 * few KB (50.4 MB), held by each GPU the library runs on until the process
 * ends.  precision: RKL_FP64 or RKL_MIXED (b double or float accordingly).
 * Limits: at most RKL_NOALLOC_MAX_CELLS cells and s_cap in [2,
 * RKL_NOALLOC_MAX_STAGES]; larger requests return RKL_EINVAL with a message.
 * s_out: device int32 (may be NULL) receiving s; if s > s_cap, T is left
 * unchanged (s_out tells).  Stencil variant 0.  Every call on one GPU shares
 * that GPU's scratch, so calls that overlap on one GPU (two streams or host
 * threads at once) race; serialise them.
 */
#define RKL_NOALLOC_MAX_CELLS 2097152   /* 2^21, e.g. 128^3 */
#define RKL_NOALLOC_MAX_STAGES 256
rkl_status rkl_superstep_noalloc(const rkl_grid_desc *grid, int32_t precision, double *T, const void *b,
                                 double dt_hyp, int32_t s_cap, int32_t *s_out, void *stream);

/*
 * rkl_subcycle: explicit sub-cycling of the conduction operator over dt_hyp
 * on one grid, T updated in place (Sec. 2.3, the sub-cycled alternative the
 * paper compares super-time-stepping with): N_sub = ceil(dt_hyp / dt_par)
 * forward-Euler sub-steps T <- T + tau (gamma-1)/rho (-div F_c(T)) with
 * tau = dt_hyp / N_sub <= dt_par, dt_par of Eq. dt_exp taken from T at the
 * start.  Reads dt_par back once (one synchronisation of `stream`); stores
 * N_sub in *nsub_out (host pointer, may be NULL; 0 when dt_hyp = 0 or there
 * is no conduction, T then unchanged).  RKL_ESTAGES (T unchanged) if N_sub
 * would exceed max_sub.  Uses one plan stage buffer as the other half of a
 * ping-pong; an odd N_sub ends with one device copy into T.
 */
rkl_status rkl_subcycle(rkl_plan_t plan, int32_t grid, double *T, const void *b, double dt_hyp,
                        int64_t max_sub, int64_t *nsub_out, void *stream);

/*
 * rkl_aag: one AAG super-time-step (Alexiades, Amiez & Gremaud 1996; the
 * first-order scheme the paper compares RKL with, Sec. 3.3) of length
 * dt_hyp on one grid, T updated in place: S forward-Euler sub-steps with the
 * damped Chebyshev sequence tau_j = dt_par / ((nu-1) cos(pi (2j-1)/(2S)) +
 * 1 + nu), j = 1..S, scaled to sum to dt_hyp, where S is the smallest count
 * whose gain (Eq. AAG-STS) reaches dt_hyp/dt_par.  nu in (0, 1) is the
 * damping.  Reads dt_par back once (one synchronisation); *s_out (host, may
 * be NULL) receives S (0: nothing to do).  RKL_ESTAGES (T unchanged) if S
 * would exceed max_s.  Same kernels and ping-pong as rkl_subcycle.
 */
rkl_status rkl_aag(rkl_plan_t plan, int32_t grid, double *T, const void *b, double dt_hyp, double nu,
                   int32_t max_s, int32_t *s_out, void *stream);

/*
 * rkl_superstep_batched: one super-step of every grid of the plan at once
 * with no host synchronisation -- safe to capture in a HIP graph: one
 * reduce launch (dt_par and s per grid on the device), then one launch per
 * stage j = 1..smax over every tile of every grid (grids with s < j skip
 * it), so the plan's smax should be the largest stage count expected.  T and b are packed
 * (grid g at rkl_grid_offset(g) cells, b at 3x that); dt_hyp is a device
 * array of ngrids doubles; s_out (device, ngrids int32, may be NULL) receives
 * each grid's stage count.  A grid whose s exceeds smax is left unchanged
 * and flagged (RKL_FLAG_STAGES, see rkl_query).
 */
rkl_status rkl_superstep_batched(rkl_plan_t plan, double *T, const void *b,
                                 const double *dt_hyp, int32_t *s_out, void *stream);

/*
 * rkl_graph_capture: record rkl_superstep_batched(plan, T, b, dt_hyp, s_out)
 * into a HIP graph owned by the plan (replacing any earlier one); nothing is
 * executed.  rkl_graph_launch replays it on `stream` (one launch per
 * super-step).  The pointers captured must stay valid while the graph is used.
 */
rkl_status rkl_graph_capture(rkl_plan_t plan, double *T, const void *b, const double *dt_hyp,
                             int32_t *s_out, void *stream);
rkl_status rkl_graph_launch(rkl_plan_t plan, void *stream);

/*
 * rkl_query: the last stage count, dt_par and flag bits (RKL_FLAG_*) computed
 * for `grid` by the last super-step, flux_div or dt_par call.  Synchronises
 * the plan's device.  Any output pointer may be NULL.
 */
rkl_status rkl_query(rkl_plan_t plan, int32_t grid, int32_t *last_s, double *last_dt_par,
                     uint32_t *flags);

/*
 * Stencil kernel variants: rkl_variant_count() of them.  rkl_variant_info
 * fills the workgroup tile (tile_x x tile_y cells, a z-chunk of tile_z
 * planes) and the stages per launch `fuse` (any pointer may be NULL):
 *   fuse 1: one RKL2 stage per launch, output tile = tile_x x tile_y;
 *   fuse F = 2, 3, 4: stages j..j+F-1 in one launch (temporal fusion of
 *           Appendix A's recurrence; 2 <= j, j+F-1 < s; the last stage, and a
 *           remainder shorter than F, run one stage per launch), output tile
 *           (tile_x-2(F-1)) x (tile_y-2(F-1)): the tile's border rings are
 *           recomputed by the neighbouring tiles.  RKL_MIXED plans of periodic
 *           3-D grids only; selecting one allocates two more FP64 stage
 *           buffers.
 * rkl_set_variant selects a variant for a plan (RKL_EINVAL if the plan
 * cannot use it, RKL_ENOMEM); the autotuner calls it.
 */
int32_t rkl_variant_count(void);
rkl_status rkl_variant_info(int32_t variant, int32_t *tile_x, int32_t *tile_y, int32_t *tile_z,
                            int32_t *fuse);
rkl_status rkl_set_variant(rkl_plan_t plan, int32_t variant);

/*
 * Kernel timing for benchmarks.  rkl_profile(plan, 1) starts recording, with
 * a pair of HIP events on the caller's stream around each stencil launch of
 * stages j >= 2 of every following rkl_superstep and (eager, not captured)
 * rkl_superstep_batched (the dominant kernels) and around each sub-step
 * launch of rkl_subcycle and rkl_aag; rkl_profile(plan, 0) stops and
 * discards.
 * rkl_profile_read synchronises and returns, over the launches of one kind
 * -- `fuse` 1: one stage per launch, 2..4: that many fused stages, 5:
 * forward-Euler sub-steps, 6: the persistent batched launch (all stages of a
 * super-step) -- the summed
 * duration in ms, the number of launches and of cell updates (batched
 * launches count 0: their work follows from the device-side stage counts).
 */
rkl_status rkl_profile(rkl_plan_t plan, int32_t enable);
rkl_status rkl_profile_read(rkl_plan_t plan, int32_t fuse, double *ms, int64_t *launches,
                            int64_t *cell_stages);

/*
 * rkl_autotune: time every stencil variant the plan can use (tile shape,
 * z-chunk, stages per launch) on `grid`
 * with the caller's fields -- `reps` super-steps of dt_hyp each, on a
 * plan-owned scratch copy of T (T itself is not modified) -- select the
 * fastest for the plan and return its index and average super-step time.
 * Allocates a scratch copy of T for the duration of the call; synchronises.
 */
rkl_status rkl_autotune(rkl_plan_t plan, int32_t grid, const double *T, const void *b, double dt_hyp,
                        int32_t reps, int32_t *best_variant, double *best_ms, void *stream);

/*
 * Tile policies of the batched launch: rkl_batch_policy_count() of them.
 * rkl_batch_policy_info gives a policy's z-chunk length (tile_z planes) and
 * whether grids wider than 32 cells are split into half-width rows
 * (half_rows 1) instead of full-width ones (any pointer may be NULL).
 * rkl_set_batch_policy selects one for a plan (policy 0 by default); a graph
 * captured before is dropped (rkl_graph_launch then returns RKL_ESTATE until
 * the next capture).  rkl_autotune_batched times `reps` batched super-steps
 * with every policy on a plan-owned scratch copy of the packed T (T itself
 * is not modified; dt_hyp is the device array of ngrids doubles), selects
 * the fastest and returns its index and average super-step time (both
 * launch modes, see rkl_set_batch_mode).  It
 * allocates the scratch for the duration of the call and synchronises.
 */
/*
 * rkl_set_batch_mode: how rkl_superstep_batched (and a graph captured from
 * it) launches a super-step.  mode 0 (default): one reduce launch, then one
 * launch per stage j = 1..smax over every tile of every grid.  mode 1: three
 * launches -- the reduce launch, a schedule launch that lists the work items
 * (stage j, grid, tile) stage after stage for the grids' device-side stage
 * counts, and one persistent launch whose workgroups take the items in list
 * order from an atomic counter; an item of stage j of a grid waits (on the
 * device) until every tile of stages 1..j-1 of that grid is done.  An item
 * only ever waits for items earlier in the list, all of them taken by running
 * workgroups, so the launch needs no co-residency guarantee; every wait is
 * bounded (2 s), and a launch that gives up sets RKL_FLAG_ABORTED (rkl_query)
 * and leaves the results invalid.  Same bits as mode 0.  mode 1 needs smax <=
 * 256 and allocates the item list (16 B x tiles x smax) on first use.  A
 * captured graph is dropped.  rkl_autotune_batched times both modes; the
 * index it returns is policy + mode x rkl_batch_policy_count().
 */
rkl_status rkl_set_batch_mode(rkl_plan_t plan, int32_t mode);
int32_t rkl_batch_policy_count(void);
rkl_status rkl_batch_policy_info(int32_t policy, int32_t *half_rows, int32_t *tile_z);
rkl_status rkl_set_batch_policy(rkl_plan_t plan, int32_t policy);
rkl_status rkl_autotune_batched(rkl_plan_t plan, const double *T, const void *b, const double *dt_hyp,
                                int32_t reps, int32_t *best_policy, double *best_ms, void *stream);

/*
 * rkl_stream: a bandwidth probe of the HBM path (not part of the method):
 * one coalesced sweep over `bytes` bytes with a given per-lane width, for
 * measuring what the stencil's loads can reach and for calibrating HBM
 * counters.  mode 0: copy src -> dst in 8-byte elements (the width of the
 * FP64 stencil loads); mode 1: copy in 16-byte elements; mode 3: copy in
 * 4-byte elements (the FP32 unit-vector loads); mode 2: read src in 8-byte
 * elements and write one double per 1024 elements read to dst (a read-only
 * sweep; dst holds bytes/8192 doubles).  bytes: a positive multiple of 16;
 * src and dst 16-byte aligned device pointers that do not overlap.
 * Enqueued on `stream`, no synchronisation.
 */
rkl_status rkl_stream(const void *src, void *dst, int64_t bytes, int32_t mode, void *stream);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *rkl_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RKL_H */
