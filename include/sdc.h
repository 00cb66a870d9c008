/*
 * sdc.h -- C ABI of the MI355X SDC reactive-flow library (libsdc.so).
 *
 * The library implements the hot path of the spectral deferred corrections
 * (SDC) update of Zingale et al., "The Castro AMR Simulation Code: Current
 * and Future Developments" (Sec. 2): the conservative split U_t = A(U) + R(U)
 * (Eq. 1) and the node-to-node correction of Eq. 2,
 *
 *   U^{m+1,(k+1)} = U^{m,(k+1)} + dt_m [A^{m,(k+1)} - A^{m,(k)}]
 *                 + dt_m [R^{m+1,(k+1)} - R^{m+1,(k)}]
 *                 + int_{t^m}^{t^{m+1}} (A^{(k)} + R^{(k)}) dt,
 *
 * whose implicit reaction part is solved per zone by Newton with an analytic
 * Jacobian.  Every computation runs in HIP kernels on the GPU.
 *
 * Conventions for every entry point:
 *  - Floating-point arrays are float64, device memory, contiguous, in
 *    structure-of-arrays layout [component][zone] with the zone index
 *    x-fastest (z = i + n0*(j + n1*k)).  Base pointers must be 8-byte aligned
 *    (256-byte alignment gives the best bandwidth).
 *  - Full states U have n_c = 2 + dim + nspec components:
 *      0: rho, 1..dim: rho u_d, dim+1: rho E, dim+2+s: rho X_s.
 *    Reacting arrays (sources R, Newton vectors) have n_r = nspec + 1
 *    components: (rho X_1 .. rho X_nspec, rho e); the last one acts on rho E.
 *  - The caller owns every array passed in; the library never frees or
 *    reallocates them.  The handle owns its own device buffers (network
 *    parameters, statistics counters, the deferred-zone queue of the Newton
 *    kernels, advection row descriptors, cached graphs, and the workspaces of
 *    the adjoint and of the split schedule, allocated on first use).
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the
 *    default stream).  The return code reports argument validation and launch
 *    errors only; device-side outcomes (unconverged or non-finite zones) are
 *    read with sdc_stats, which synchronises.
 *  - Functions never abort or throw across the ABI.  On failure they return a
 *    nonzero SDC_ERR_* code and sdc_last_error describes it.
 *  - A handle is not thread-safe and serves one stream at a time.
 */
#ifndef SDC_H
#define SDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SDC_OK 0
#define SDC_ERR_ARG 1         /* invalid argument or configuration */
#define SDC_ERR_HIP 2         /* a HIP runtime call failed */
#define SDC_ERR_NOMEM 3       /* device allocation failed */
#define SDC_ERR_NEWTON 4      /* sdc_check: some solves did not converge (outputs written, flagged) */
#define SDC_ERR_NONFINITE 5   /* sdc_check: some solves gave non-finite results */
#define SDC_ERR_UNSUPPORTED 6 /* configuration outside the supported range */
#define SDC_ERR_COMPILE 7     /* run-time compilation of the kernels failed */

#define SDC_FP64 0  /* every step in float64 */
#define SDC_MIXED 1 /* Newton matrix and LU in float32; residual, update, quadrature in float64 */

#define SDC_MAX_NODES 5  /* temporal nodes per step: 2..5 */
#define SDC_NODES_LOBATTO 0
#define SDC_NODES_RADAU 1
#define SDC_MAX_SPECIES 31

/* counters returned by sdc_stats */
#define SDC_STAT_HIST 0       /* [0..15]: solves by Newton iteration count (15 = 15 or more) */
#define SDC_STAT_FAILED 16    /* solves that did not converge within newton_maxiter */
#define SDC_STAT_ITERS 17     /* total Newton iterations of converged solves */
#define SDC_STAT_NONFINITE 18 /* solves whose result is not finite */
#define SDC_STAT_SOLVES 19    /* zone solves */
#define SDC_STAT_FALLBACK 20  /* Newton iterations that took the pivoted dense path */
#define SDC_NSTATS 21

typedef struct sdc_handle_s* sdc_handle;

/*
 * Reaction network (host memory, copied by sdc_init).  Synthetic Arrhenius
 * kinetics on x = (rho X, rho e) with T = (gamma - 1) x_e / rho:
 *   k_r = exp(lnA_r + b_r ln T - E_r / T)
 *   v_r = k_r x_a (unimolecular)  or  k_r x_a x_c (bimolecular)
 *   R_i = sum_r stoich[r][i] v_r,  R_e = sum_r Q_r v_r,  Q_r = -sum_i stoich[r][i] q_i.
 * The paper's network is a stiff nuclear network (Sec. 2, Sec. 4); this one is
 * drawn from a seed and carries no physical data.
 */
typedef struct {
  int32_t nspec;             /* species, 1..SDC_MAX_SPECIES */
  int32_t nreact;            /* reactions, >= 0 */
  const int32_t* reactants;  /* [nreact][2] reactant species; second = -1 for unimolecular */
  const double* stoich;      /* [nreact][nspec] stoichiometric coefficients (mass units) */
  const double* lnA;         /* [nreact] */
  const double* b;           /* [nreact] temperature exponents */
  const double* E;           /* [nreact] activation temperatures */
  const double* q;           /* [nspec] specific binding energies */
} sdc_network;

/* Grid, method and solver settings (host memory, copied by sdc_init). */
typedef struct {
  int32_t dim;             /* 1, 2 or 3 */
  int64_t n[3];            /* zones per direction (x, y, z); entries beyond dim ignored */
  double dx[3];            /* zone widths; the grid is periodic in every direction */
  double gamma;            /* gamma-law EOS, p = (gamma - 1) rho e, code units p = rho T */
  int32_t n_nodes;         /* temporal nodes per step, 2..5 (Gauss-Lobatto: 2 = trapezoid, 3 = Simpson) */
  int32_t n_iters;         /* SDC iterations K per step, >= 1 */
  int32_t precision;       /* SDC_FP64 or SDC_MIXED */
  int32_t advection;       /* 0: A == 0 (reaction only), 1: advective term on */
  int32_t slope;           /* 0: central slopes, 1: monotonized-central slopes */
  double alpha;            /* > 0: frozen Rusanov speed; <= 0: local max(|u| + c) */
  double newton_tol;       /* Newton stops when its scaled step e_k = max_i |delta_i| / s_i
                            * (s = rho, |b_e|) is <= tol, or when e_k < e_{k-1} and
                            * e_k^2 / (e_{k-1} - e_k) <= tol (the contraction bounds the
                            * distance of the new iterate from the root by tol) */
  int32_t newton_maxiter;  /* >= 1 */
  double pivot_threshold;  /* tau: a pivot below tau * column max takes the pivoted path */
  /* Batched boxes: nbox > 0 replaces the single grid by nbox independent
   * periodic boxes sharing dx (n[] is ignored).  box_n (host, copied) holds
   * [nbox][3] extents (x, y, z; entries beyond dim ignored).  The state is the
   * concatenation of the boxes in order, each box x-fastest, still SoA
   * [component][zone] over all zones. */
  int32_t nbox;
  const int64_t* box_n;
  /* 1: sdc_step replays one captured HIP graph per step (per buffer-rotation
   * phase); 0 (default): plain launches.  Profiling forces launches. */
  int32_t graph;
  /* 1: the first sdc_step call takes the schedule cached on disk for this
   * kernel source and size, or runs sdc_autotune on its input; 0 (default):
   * the schedule set with sdc_set_schedule (initially 0, 0, 0, 0). */
  int32_t autotune;
  /* Temporal nodes of a step (n_nodes of them, tau_0 = 0 and tau_M = 1):
   * SDC_NODES_LOBATTO (default): Gauss-Lobatto points, the node-to-node
   * integrals interpolate through every node (trapezoid and Simpson for 2 and
   * 3 nodes, Sec. 2); SDC_NODES_RADAU: tau_0 = 0 followed by the n_nodes - 1
   * right Radau points, the integrals interpolate through the Radau points
   * only, so the sweeps converge to Radau IIA collocation, which damps very
   * stiff modes (the quadratures for highly stiff reactions of Sec. 5). */
  int32_t node_type;
  /* Spatial order of the finite-volume terms: 2 (default; PLM + Rusanov as
   * above, zone-local sources) or 4, the paper's fourth-order method (Sec. 2:
   * Simpson in time with McCorquodale and Colella's reconstruction): A from
   * fourth-order face averages, face-centre values and face-averaged fluxes
   * (no limiter, so slope and alpha are ignored; for smooth flows), and the
   * reactive terms as zone averages of R at zone-centre states, the Newton
   * solve of each transition running on the zone-centre values of its
   * right-hand side.  Single grids only (nbox = 0); no adjoint. */
  int32_t space_order;
} sdc_config;

/*
 * Caller-owned node arrays for sdc_sweep / sdc_step, M = n_nodes - 1:
 *   U[0..M]  [n_c][Z]  states at the nodes
 *   A[0..M]  [n_c][Z]  advective terms at the nodes
 *   R[0..M]  [n_r][Z]  reactive sources at the nodes
 *   C[0..M-2][n_c][Z]  correction terms of transitions 1..M-1 (scratch)
 * Unused entries may be NULL.  Distinct entries must not overlap.
 */
typedef struct {
  double* U[SDC_MAX_NODES];
  double* A[SDC_MAX_NODES];
  double* R[SDC_MAX_NODES];
  double* C[SDC_MAX_NODES - 2];
} sdc_nodes;

/*
 * Two-level hierarchy: refined patches with subcycling in time around the
 * SDC step (the extension to adaptive mesh refinement that Sec. 2 and Sec. 5
 * name).  Level 0 is the periodic coarse grid of `coarse`; every patch is a
 * box of coarse zones (lo, ext per direction, x y z; inside the grid, two or
 * more coarse zones from every other patch and from itself, also across the
 * periodic boundary) refined by 2 in space and time.
 * Patch arrays are padded by 2 ghost zones per side and concatenated in patch
 * order, each x fastest, SoA [n_c][Zf] (the layout of batched boxes with
 * extents 2 ext + 4).  A coarse step of length dt: the coarse level takes one
 * SDC step on every zone; each patch takes two steps of dt / 2 whose ghost
 * zones are filled before every evaluation of A from the coarse node states
 * of this step's last iteration (Lagrange polynomial through the node times
 * in time, conservative piecewise-linear with central coarse slopes in space),
 * with A zero in the ghost zones; the time-integrated fluxes of the last
 * sweep through the coarse-fine faces are accumulated on both levels; the
 * uncovered coarse zones next to a patch are refluxed with the averaged fine
 * fluxes, and every covered coarse zone takes the mean of its fine zones.
 * Composite-grid mass, momentum and total energy are conserved to rounding.
 * Requirements: nbox = 0 and space_order = 2 in `coarse`.  Errors of
 * sdc_amr_create come from sdc_last_error(NULL); later errors from
 * sdc_last_error of the coarse handle (sdc_amr_handles).
 */
typedef struct sdc_amr_s* sdc_amr;
typedef struct {
  int32_t npatch;
  const int64_t* lo;   /* [npatch][3] first covered coarse zone (x, y, z; entries beyond dim ignored) */
  const int64_t* ext;  /* [npatch][3] covered coarse zones per direction */
} sdc_patches;

int sdc_amr_create(const sdc_config* coarse, const sdc_network* net, const sdc_patches* patches, sdc_amr* out);
int sdc_amr_destroy(sdc_amr a);
/* Zones of the coarse grid and of all padded patches together. */
int sdc_amr_sizes(sdc_amr a, int64_t* zc, int64_t* zf);
/* The two handles (coarse, and the patches as batched boxes): statistics,
 * profiling and errors of the levels.  Owned by the hierarchy. */
int sdc_amr_handles(sdc_amr a, sdc_handle* coarse, sdc_handle* fine);
/* Every patch zone, ghosts included, from the coarse state Uc by the
 * conservative piecewise-linear interpolation (initial data).  Synchronises. */
int sdc_amr_fill_patches(sdc_amr a, const double* Uc, double* Uf, void* stream);
/* nsteps coarse steps of length dt; Uc [n_c][Zc] and Uf [n_c][Zf] are
 * updated in place (node arrays are owned by the hierarchy). */
int sdc_amr_step(sdc_amr a, double dt, int32_t nsteps, double* Uc, double* Uf, void* stream);

/* Fill `cfg` with defaults: 3 nodes, K = 4, FP64, MC slopes, local Rusanov
 * speed, gamma 1.4, tol 1e-13, maxiter 50, pivot threshold 0.1, no boxes,
 * plain launches. */
int sdc_config_default(sdc_config* cfg);

/*
 * Create a handle: validates the configuration, generates the network's
 * device code (rates, residual, packed Newton matrix and its fixed-order LU)
 * and compiles it with the kernels for gfx950 (cached on disk, see
 * SDC_KERNEL_CACHE), uploads the network parameters.  3D grids take the row
 * advection kernel where their rows fit a block; SDC_ADVECT_ROWS=0 in the
 * environment selects the zone-per-thread kernel instead (same fluxes, for
 * comparison).
 * Errors: SDC_ERR_ARG, SDC_ERR_UNSUPPORTED, SDC_ERR_COMPILE, SDC_ERR_HIP,
 * SDC_ERR_NOMEM.  On error *out is NULL; sdc_last_error(NULL) explains.
 */
int sdc_init(const sdc_config* cfg, const sdc_network* net, sdc_handle* out);

/* Release the handle and its device buffers (synchronises its work first). */
int sdc_destroy(sdc_handle h);

/* Description of the last error on `h` (or of the calling thread's last
 * sdc_init failure when h is NULL).  Owned by the library. */
const char* sdc_last_error(sdc_handle h);

/* Zones Z, components n_c and reacting components n_r of the handle's grid. */
int sdc_sizes(sdc_handle h, int64_t* zones, int32_t* ncomp, int32_t* nreact_vars);

/*
 * A = <A(U)>: the advective term of Eq. 1 on the periodic grid, the negative
 * divergence of Rusanov fluxes of a piecewise-linear reconstruction of the
 * conserved variables (method of lines).  U, A: [n_c][Z]; must not overlap.
 */
int sdc_advective_term(sdc_handle h, const double* U, double* A, void* stream);

/* R = R(U): the reactive source of Eq. 1 on the reacting components,
 * evaluated at x = (rho X, rho E - |rho u|^2 / (2 rho)).  U: [n_c][Z], R: [n_r][Z]. */
int sdc_source(sdc_handle h, const double* U, double* R, void* stream);

/*
 * The implicit part of Eq. 2 alone, per zone: solve x - dt_m R(x; rho) = b by
 * Newton from the guess in x.  rho: [Z]; b, x, R: [n_r][Z]; iters: int32 [Z].
 * Outputs: x = root, R = R(x), iters = Newton iterations or -1 (not converged
 * within newton_maxiter; x keeps the last iterate).  x and b must not overlap.
 */
int sdc_reaction_solve(sdc_handle h, double dt_m, const double* rho, const double* b, double* x,
                       double* R, int32_t* iters, void* stream);

/*
 * sdc_reaction_solve for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, on `nzones` zones of arrays laid
 * out [component][nzones] (rho: [nzones]; b, x, R: [n_r][nzones]; iters:
 * int32 [nzones]), independent of the handle's grid size.  Its deferred-zone
 * queue lives in a fixed device array of SDC_NOALLOC_SCRATCH_BYTES inside the
 * library (one per device, held until the process ends), so the call makes no
 * hipMalloc, hipFree or other allocation and records no profiling events.
 * Limit: the queue needs 28 + 16 n_r bytes per zone (plus at most 2 KiB of
 * alignment), about 266,000 zones at n_r = 14; a larger nzones returns
 * SDC_ERR_ARG (the message gives the limit).  nzones = 0 is a no-op.  Calls that overlap on
 * one device (concurrent streams, or handles on several threads) share that
 * device's array and race; calls serialised on one stream do not.  The queue
 * counter is cleared by a kernel at the start of each call.  Errors as
 * sdc_reaction_solve, plus SDC_ERR_HIP if the array's address could not be
 * resolved when the handle was created.
 */
#define SDC_NOALLOC_SCRATCH_BYTES (64ll << 20)
int sdc_reaction_solve_noalloc(sdc_handle h, double dt_m, int64_t nzones, const double* rho, const double* b,
                               double* x, double* R, int32_t* iters, void* stream);

/*
 * One SDC iteration k -> k+1 over the transitions m = 0..M-1 of Eq. 2 for a
 * step of length dt, followed by A at the last node.  On entry nodes->U[0],
 * A[0], R[0] hold U^n, A(U^n), R(U^n); for k >= 1 the other nodes hold
 * iteration k; for k == 0 every iteration-0 node is taken to equal node 0
 * (entries 1..M are not read).  On return nodes 1..M hold iteration k+1.
 */
int sdc_sweep(sdc_handle h, double dt, int32_t k, const sdc_nodes* nodes, void* stream);

/*
 * nsteps SDC steps of length dt, each of n_iters sweeps; U [n_c][Z] holds
 * U^n on entry and the final state on return (U^{n+1} = U^{M,(K)}).  `work`
 * supplies the node arrays (U, A, R for every node and C when M >= 2); none
 * of them may overlap U.  The last node's A and R carry over as node 0 of the
 * next step.
 */
int sdc_step(sdc_handle h, double dt, int32_t nsteps, double* U, const sdc_nodes* work, void* stream);

/* Copy the accumulated counters (SDC_STAT_*) to host `out[SDC_NSTATS]`;
 * synchronises the handle's last stream. */
int sdc_stats(sdc_handle h, int64_t* out);

/* Device-side outcome of the work since the last sdc_stats_reset, as a
 * status: synchronises like sdc_stats, then returns SDC_ERR_NONFINITE if any
 * solve gave a non-finite result, else SDC_ERR_NEWTON if any solve stopped
 * at newton_maxiter without converging (its zone kept the last iterate and
 * its iteration count reads -1), else SDC_OK.  sdc_last_error gives the
 * counts.  Launch-time entry points never return these two codes: they
 * enqueue work whose outcome is known only after it ran. */
int sdc_check(sdc_handle h);

/* Zero the counters (enqueued on `stream`). */
int sdc_stats_reset(sdc_handle h, void* stream);

/* Replace the rate parameters lnA and E (host arrays [nreact]); enqueued on
 * the handle's last stream before any later work. */
int sdc_set_params(sdc_handle h, const double* lnA, const double* E);

/*
 * Adjoint of one step (reverse mode): given U^n and the adjoint Ubar^{n+1} of
 * the step's output U^{n+1}, writes Ubar^n = (dU^{n+1}/dU^n)^T Ubar^{n+1} and
 * accumulates thetabar[0..nreact) += d/dlnA_r, thetabar[nreact..2 nreact) +=
 * d/dE_r of (Ubar^{n+1} . U^{n+1}).  The step is replayed forward from U^n
 * (node states of every iteration kept in handle-owned workspace, allocated
 * on first use), then every implicit reaction solve is differentiated with
 * the implicit-function theorem at its converged root and the quadrature and
 * advective terms are transposed.  Requires a single grid and, with
 * advection on, the smooth mode (slope 0, frozen alpha > 0); otherwise
 * SDC_ERR_UNSUPPORTED.  U_n, Ubar_np1, Ubar_n: [n_c][Z] device, distinct;
 * thetabar: device [2 nreact].  Deterministic: no floating-point atomics.
 */
int sdc_step_adjoint(sdc_handle h, double dt, const double* U_n, const double* Ubar_np1, double* Ubar_n,
                     double* thetabar, void* stream);

/*
 * Kernel schedule of the node transitions: occ2 = 1 selects the Newton
 * variants built for two wavefronts per SIMD (smaller register budget), occ2
 * = 0 the compiler's budget; cap > 0 stops the fast Newton pass after `cap`
 * iterations and finishes the zones still unconverged in a second kernel,
 * which packs the slow tail of the Newton counts into dense wavefronts (cap =
 * 0: no cap); split > 0 cuts every transition into `split` zone batches whose
 * explicit part (quadrature, rhs) runs in its own kernel on a second stream
 * beside the Newton kernel of the previous batch (split = 0: one fused kernel
 * per transition; captured steps always use the fused kernels); zchunk > 0
 * sets the tile of the 3D row advection kernel, the number of z planes one
 * row marches (0: chosen from the grid size).  Every schedule produces
 * bitwise-identical results.  Returns SDC_ERR_ARG for occ2 outside {0, 1},
 * cap < 0, split outside [0, 64] or zchunk outside [0, 1024].  A new zchunk
 * synchronises the handle's last stream (the tile table is rewritten).
 */
int sdc_set_schedule(sdc_handle h, int32_t occ2, int32_t cap, int32_t split, int32_t zchunk);
int sdc_get_schedule(sdc_handle h, int32_t* occ2, int32_t* cap, int32_t* split, int32_t* zchunk);

/*
 * Time every fused schedule (occ2 in {0,1} x cap in {0,2,3,4,5,6}, split 0) on
 * one SDC step from U (read only; `work` is scratch) with HIP events on
 * `stream`, then the row-kernel tile (zchunk in {0, 16, 32, 64, 128}) on the
 * advective term of U; keep the fastest of each (the defaults unless another
 * is faster by more than 1%), and cache the choice on disk per kernel source
 * and zone count.  Newton statistics are left unchanged.  Synchronises.
 */
int sdc_autotune(sdc_handle h, double dt, const double* U, const sdc_nodes* work, void* stream);

/* Kernel kinds for sdc_profile_read. */
#define SDC_K_ADVECT 0
#define SDC_K_SOURCE 1
#define SDC_K_SOLVE 2
#define SDC_K_TRANSITION_FIRST 3
#define SDC_K_TRANSITION_NODE0 4
#define SDC_K_TRANSITION_LATER 5
#define SDC_K_FILL 6
#define SDC_K_ADJOINT 7  /* every kernel of the adjoint pass */
#define SDC_K_FINISH 8   /* second-stage kernels of capped or guarded Newton solves */
#define SDC_K_SPLIT 9    /* batch kernels of the split schedule (each transition is also timed as one span) */
#define SDC_K_ORDER4 10  /* centre conversions and average stores of fourth-order transitions */
#define SDC_NKINDS 11

/*
 * Per-kernel timing: while enabled, every launch is bracketed by HIP events
 * recorded on the launch stream.  sdc_profile_read synchronises, returns the
 * summed milliseconds and launch counts per kernel kind (SDC_K_*; arrays of
 * SDC_NKINDS) since the last read, and clears them.
 */
int sdc_profile_enable(sdc_handle h, int32_t enable);
int sdc_profile_read(sdc_handle h, double* ms, int64_t* launches);

/*
 * Operation counts of the generated network code (add, mul, div, exp and log
 * count 1, fused multiply-add 2): out[0] R(x), out[1] residual and Newton
 * matrix, out[2] LU factorisation, out[3] triangular solves, out[4] exp calls
 * per evaluation, out[5] structural nonzeros of the Newton matrix, out[6]
 * with fill-in.
 */
int sdc_cost_model(sdc_handle h, int64_t* out);

/*
 * Compile (or find in the cache) the kernels for `cfg` and `net` without
 * touching a GPU; for build steps that warm the kernel cache.
 */
int sdc_compile_only(const sdc_config* cfg, const sdc_network* net);

/* Path of the ahead-of-time code object for `cfg` and `net` in the kernel
 * cache directory (SDC_KERNEL_CACHE, else _kcache beside the library).  A
 * build step may place there the generated source compiled with hipcc
 * --genco and the options of the run-time compiler; sdc_init then loads it
 * instead of compiling with hipRTC.  Copies up to `len` bytes including the
 * terminator into `buf` and returns the full length needed, or a negative
 * SDC_ERR_* code. */
int64_t sdc_aot_name(const sdc_config* cfg, const sdc_network* net, char* buf, int64_t len);

/* Generated device source for `cfg` and `net` (for inspection): copies up to
 * `len` bytes including the terminator into `buf` and returns the full length
 * needed, or a negative SDC_ERR_* code. */
int64_t sdc_generated_source(const sdc_config* cfg, const sdc_network* net, char* buf, int64_t len);

#ifdef __cplusplus
}
#endif
#endif /* SDC_H */
