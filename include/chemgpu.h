/*
 * chemgpu.h -- C ABI of the MI355X (gfx950) per-cell chemistry integrator.
 *
 * The library advances, for every cell independently, the chemistry ODE of
 * the paper's reactive part (Sec. 2.2.3, Eq. 20): u = (T, Y_1..Y_N) at
 * constant density and internal energy, with species sources from
 * mass-action kinetics (Sec. 2.1.2, Eq. 14-16; Arrhenius forward rates,
 * reverse rates from NASA-7 equilibrium constants, optional third-body
 * efficiencies), over one flow time step dt, using the five-stage
 * fourth-order low-storage explicit Runge-Kutta scheme in the two-register
 * form of Eq. 21 with an embedded third-order error register and the WRMS
 * step-size controller of Eq. 22 (factor clamp [1/5, 5], safety 0.9).
 *
 * All arithmetic of the integrator is FP64.  Every entry point that takes a
 * `stream` enqueues on that HIP stream (a hipStream_t passed as void*, NULL =
 * the null stream) and returns without synchronising unless stated.
 *
 * Errors: every int-returning call returns CHEM_OK (0) or a negative code
 * below; chem_last_error() gives a message for the calling thread's last
 * failure.  Per-cell outcomes never fail a call: they go to the status array.
 * Handles are not thread-safe; calls on one handle must not overlap.
 *
 * Device memory: the integration calls (chem_integrate, chem_integrate_batched,
 * chem_react_conserved, surrogate_infer, chem_integrate_noalloc) allocate
 * nothing and never synchronise the device (chem_integrate_batched's host
 * wait on its staging ring is described there).  Their workspace is
 * allocated up front by chem_workspace_reserve (and surrogate_reserve); a
 * call on more cells than the reservation holds returns CHEM_ECAPACITY and
 * enqueues nothing.  Only the set-up calls allocate: chem_workspace_reserve,
 * surrogate_create/reserve/train/grad/forward, chem_autotune,
 * surrogate_autotune, chem_graph_capture_batched and surrogate_graph_capture.
 */
#ifndef CHEMGPU_H
#define CHEMGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define CHEM_OK 0
#define CHEM_EINVAL (-1)       /* null pointer, n < 0, ld < n, dt <= 0, bad option */
#define CHEM_ENOMEM (-2)       /* device or host allocation failed */
#define CHEM_EHIP (-3)         /* a HIP runtime call failed (message has the HIP error) */
#define CHEM_EPARSE (-4)       /* mechanism file unreadable or malformed (message has the line) */
#define CHEM_EUNSUPPORTED (-5) /* no kernel was built for this mechanism's content hash */
#define CHEM_ECAPACITY (-6)    /* more cells (or boxes) than the reserved workspace holds */

/* Per-cell status codes written to the status array. */
#define CHEM_CELL_OK 0          /* reached dt */
#define CHEM_CELL_MAXSTEPS 1    /* step budget (accepted + rejected) exhausted before dt */
#define CHEM_CELL_NONFINITE 2   /* non-finite input; the cell was left unchanged */
#define CHEM_CELL_H_UNDERFLOW 3 /* step size fell below 1e-14 * dt */
#define CHEM_CELL_T_NEWTON 4    /* chem_react_conserved: no temperature for the cell's energy */

typedef struct chem_mech_s *chem_mech; /* opaque, owned by the library */

/* Integration options; a zero field selects the default. */
typedef struct {
    double rtol;         /* relative tolerance of Eq. 22 (default 1e-8) */
    double atol;         /* absolute tolerance of Eq. 22, every component (default 1e-10) */
    int32_t max_steps;   /* accepted + rejected steps per cell (default 100000) */
    int32_t chunk_steps; /* steps a lane takes between compaction points; 0 = tuned default,
                            < 0 = no compaction (one cell per lane for the whole step) */
    int32_t block_size;  /* threads per block, multiple of 64 up to 512 (0 = tuned default) */
    int32_t fixed_steps; /* > 0: test mode, exactly this many steps of dt/fixed_steps, no control */
    int32_t tail_steps;  /* a cell still stepping after this many steps (accepted + rejected,
                            over all sub-calls) is handed over; if at most tail_cap cells
                            per CU are handed over they are finished by the cooperative
                            kernel, several lanes per cell, otherwise one cell per lane as
                            before.  0 = tuned default, < 0 = never.  The hand-off point and
                            that choice depend only on the input, so results do not depend
                            on block_size or chunk_steps */
    int32_t scheme;      /* 0: the paper's low-storage LSRK4(3)5 two-register scheme (Eq. 21);
                            1: the full-storage Runge-Kutta-Fehlberg 4(5) comparison scheme
                            (six stages, all stage vectors kept; same controller with
                            exponent 1/5; no cooperative tail);
                            2: the implicit comparator, a fourth-order Rosenbrock method
                            (Shampine's parameters, Kaps-Rentrop form, embedded third
                            order; exact Jacobian, LU with partial pivoting; same
                            controller, exponent 1/4; no cooperative tail).  Built only for
                            mechanisms of at most 15 species (CHEM_EUNSUPPORTED otherwise)
                            and run with block_size <= 256 (CHEM_EINVAL otherwise) */
    int32_t tail_cap;    /* most handed-over cells per CU that the cooperative kernel takes
                            (see tail_steps): 0 = the tuned value (64 when none is tuned),
                            > 0 = that many, < 0 = no limit */
    int32_t pool_order;  /* 1: before the step, cells expected to take many steps (a step
                            hint below dt/8 over the flow step, or without a usable hint
                            T >= 1000 K) are dealt round-robin over the first work claim of
                            every resident block, so they start at once and spread over the
                            chip; 2: cells below the mechanism's NASA-7 range switch (the
                            T_mid most species share) come first, the others after them,
                            so that few waves hold cells of both ranges (such a wave
                            evaluates both sets of polynomials); 3: as 2, and with a
                            hand-off point (tail_steps) the first launch takes only the
                            cells above the switch: the others are stepped by the
                            per-lane resumption after its tail list, where they fill
                            the lanes its longest cells leave idle (without a hand-off
                            point, as 2); < 0: pool order as laid out; 0: tuned
                            default, else off; > 3: CHEM_EINVAL.  Changes no result
                            (cells are independent); uses 8 bytes of workspace per
                            cell */
} chem_opts;

/*
 * State layout (every entry point): structure of arrays of doubles in device
 * memory, state[v * ld + i] for cell i < n_cells and row v:
 *   v = 0        T    [K]                      in/out
 *   v = 1..N     Y_k  mass fractions            in/out
 *   v = N+1      rho  [g/cm^3]                  in (constant over the step)
 *   v = N+2      h    step-size hint [s]        in (<= 0 or >= dt: start with dt) /
 *                                               out (controller's next proposal)
 * with ld >= n_cells.  The caller owns the memory.
 */

/* Load a mechanism from a .mech text file and bind the kernel that was
 * generated for it at build time, keyed by the FNV-1a 64 hash of the file's
 * bytes.  *out receives a handle to free with chem_mech_free.  The handle
 * belongs to the device current at this call (every later call on it must
 * run with that device current); the first load on a device also looks up
 * that device's address of chem_integrate_noalloc's scratch array.  Allocates
 * no device memory (see chem_workspace_reserve). */
int chem_mech_load(const char *path, chem_mech *out);

/* Species count N, reaction count and content hash of a loaded mechanism. */
int chem_mech_query(chem_mech m, int32_t *n_species, int32_t *n_reactions, uint64_t *hash);

/* Release a mechanism and its workspace (destroy its graphs first). */
void chem_mech_free(chem_mech m);

/* Allocate the mechanism handle's whole device workspace for calls on up to
 * max_cells cells (all boxes of a batched call together): the work-pool
 * counter, a ring of 4 box tables of 4096 entries (device memory plus a
 * pinned host staging copy), the tail records through which the per-lane
 * kernel hands long-running cells to the cooperative kernel or its own
 * resumption (the cell's state and progress, N+7 doubles rounded up to a
 * multiple of 64 bytes, plus 8 B of sort key and order per cell), the pool
 * order (8 B per cell) and chem_react_conserved's primitive work state
 * ((N+3) doubles + 1 byte per cell): 241 B per cell for 9 species.
 * This is the only call that allocates for chem_integrate,
 * chem_integrate_batched and chem_react_conserved; past the reservation they
 * return CHEM_ECAPACITY.  A reservation never shrinks; growing one first
 * waits for the whole device (hipDeviceSynchronize), since queued calls may
 * still use the old buffers.  max_cells = 0 allocates only the fixed part.
 * CHEM_EINVAL for a null handle or max_cells < 0; CHEM_EHIP if an allocation
 * fails (the per-cell part is then released and the reservation is 0). */
int chem_workspace_reserve(chem_mech m, int64_t max_cells);

/*
 * Per-kernel timing (for measurement, not needed to integrate).  With on != 0
 * every later chem_integrate / chem_integrate_batched / chem_react_conserved
 * call on m records HIP events on its stream around each launch of the flow
 * step, and so does surrogate_infer with fallback around the FP64 run of the
 * cells outside the training hull, on its side stream (creating the events
 * on first use; captured graphs and chem_integrate_noalloc are not timed);
 * on == 0 stops it.  chem_kernel_times then waits for the last such call and
 * writes n >= 4 durations in ms: [0] the persistent per-lane kernel, [1] the
 * tail-list sort, [2] the cooperative kernel, [3] the per-lane resumption of
 * the tail list, and with n >= 5 [4] the whole flow step (0 for what the
 * call did not launch).  chem_tail_stats waits the same way and
 * writes n >= 3 counts of that call: [0] cells handed over to the tail list,
 * [1] of them finished by the cooperative kernel, [2] the steps (accepted +
 * rejected) the cooperative kernel took.  CHEM_EINVAL for a null argument, n
 * too small, or no timed call since timing was last set.
 */
int chem_set_kernel_timing(chem_mech m, int32_t on);
int chem_kernel_times(chem_mech m, float *ms, int32_t n);
int chem_tail_stats(chem_mech m, int64_t *out, int32_t n);

/*
 * Advance n_cells cells by dt (paper Eq. 20-22), in place.
 *   status: NULL or int32[n_cells] device array of CHEM_CELL_* codes.
 *   counts: NULL or int32[2 * n_cells] device array; counts[i] = accepted
 *           steps, counts[n_cells + i] = rejected steps of cell i.
 * Enqueued on `stream`; no host synchronisation, no allocation.
 * CHEM_ECAPACITY if n_cells exceeds the reservation (chem_workspace_reserve),
 * except with chunk_steps < 0 (one cell per lane, no workspace).
 */
int chem_integrate(chem_mech m, double *state, int64_t ld, int64_t n_cells, double dt,
                   const chem_opts *opts, void *stream, int32_t *status, int32_t *counts);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * flow step as chem_integrate, same arguments, results and per-cell outputs,
 * bitwise equal, with no allocation and no workspace reservation.  Its
 * scratch memory (work-pool counter, tail records, pool order) is a fixed
 * device array inside the library, one copy per GPU, sized for at most
 * 1,048,576 cells (46 MB, held from the first chem_mech_load on that GPU
 * until the process ends); CHEM_ECAPACITY for more cells.  Every call on one
 * GPU shares that array, whatever the handle: calls that overlap on one GPU
 * (two streams, or two host threads) race and give wrong results.  Each call
 * clears the counters it uses (kernels, no memset) before its integration.
 * Enqueued on `stream`; no host synchronisation.
 */
int chem_integrate_noalloc(chem_mech m, double *state, int64_t ld, int64_t n_cells, double dt,
                           const chem_opts *opts, void *stream, int32_t *status, int32_t *counts);

/*
 * The reaction step of an operator-split flow solver (paper Sec. 2.2.1: the
 * Strang split applies this for dt/2, the hydrodynamic step for dt, and
 * this for dt/2 again), on the flow solver's conserved variables, in place.
 * Structure of arrays of doubles, cons[v * ld + i], rows:
 *   0 rho, 1..3 rho u, rho v, rho w, 4 rho E (total energy per volume,
 *   internal + kinetic, cgs), 5..4+N rho Y_k, 5+N T [K] (in: Newton initial
 *   guess, <= 0 => 1000 K; out: temperature after the step), 6+N h (step
 *   hint, as in chem_integrate).
 * Per cell: Y = rho Y / rho; T from e = E - |u|^2/2 by Newton iteration on
 * the mixture internal energy of the NASA-7 fits (|dT| <= 1e-12 T within 50
 * iterations, else status CHEM_CELL_T_NEWTON and the cell is left unchanged);
 * the chemistry ODE over dt at constant rho and e (as chem_integrate); then
 * rho Y_k, T and h are written back.  rho, momentum and rho E are not
 * touched (the step conserves them).  Uses the primitive work state of
 * (N+3) doubles per cell that chem_workspace_reserve allocates;
 * CHEM_ECAPACITY if n_cells exceeds the reservation.  status / counts as in
 * chem_integrate.  Enqueued on `stream`; no host synchronisation.
 */
int chem_react_conserved(chem_mech m, double *cons, int64_t ld, int64_t n_cells, double dt,
                         const chem_opts *opts, void *stream, int32_t *status, int32_t *counts);

/*
 * One AMR box (block-structured patch) of a batched call.  The box's cells
 * are advanced by n_sub successive sub-calls of dt each -- a level-l box of
 * a hierarchy with refinement ratio r takes r^l sub-steps of dt_0 / r^l per
 * coarse step (paper Sec. 3.2, Algorithm 1) -- carrying the step-size hint
 * between sub-calls.  max_steps applies to each sub-call; counts accumulate
 * over them; the first sub-call that ends with a non-OK status stops the cell.
 */
typedef struct {
    double *state;   /* SoA block as above, caller-owned device memory */
    int64_t ld;      /* leading dimension, >= n_cells */
    int64_t n_cells; /* cells in the box (>= 0) */
    double dt;       /* sub-call length for this box's level [s], > 0 */
    int32_t n_sub;   /* sub-calls (>= 1) */
    int32_t level;   /* refinement level (informational; used to order work) */
    int32_t *status; /* NULL or int32[n_cells] device array */
    int32_t *counts; /* NULL or int32[2 * n_cells] device array (accepted, rejected) */
} chem_box;

/*
 * Advance every cell of n_boxes boxes in ONE persistent launch over a shared
 * work pool: deeper-level boxes (more sub-calls) are queued first, still-active
 * cells are compacted within each workgroup between step chunks.  The box
 * table is copied to the device through one slot of the handle's ring of 4
 * pinned staging tables; a slot is reused once the batched call that used it
 * last has finished on the device, so the host waits only when 4 earlier
 * batched calls on this handle are still queued.  CHEM_ECAPACITY if the
 * boxes hold more cells than the reservation or more than 4096 of them are
 * non-empty.
 */
int chem_integrate_batched(chem_mech m, const chem_box *boxes, int32_t n_boxes,
                           const chem_opts *opts, void *stream);

typedef struct chem_graph_s *chem_graph; /* opaque, owned by the library */

/*
 * Capture a batched call into a HIP graph (reset kernel + persistent
 * kernel; no memset nodes).  The box table is copied to graph-owned device
 * memory at capture time, so every later launch integrates the same boxes
 * (same pointers, sizes, dt, n_sub) with whatever data they then hold.
 * Capture happens on a private stream (`stream` may be NULL and is only
 * synchronised before the capture).  The graph has its own work-pool
 * counter, so it may be launched while eager calls use the mechanism on the
 * same stream; two launches of one graph must not overlap.  Allocates (at
 * capture time only).
 */
int chem_graph_capture_batched(chem_mech m, const chem_box *boxes, int32_t n_boxes,
                               const chem_opts *opts, void *stream, chem_graph *out);

/* Launch a captured graph on `stream` (enqueue only). */
int chem_graph_launch(chem_graph g, void *stream);

/* Destroy a graph (waits for its outstanding launches). */
void chem_graph_destroy(chem_graph g);

/*
 * Autotune block size, chunk length and cooperative hand-off for these
 * boxes by coordinate descent: chunk in {1, 2, 4, 8, 16, 32, 64} at the
 * default block, then, when the best of those calls took under 50 ms,
 * every pair of block in {64, 128, 192, 256, 384, 512} (those that fit the
 * LDS compaction slots) and chunk, otherwise block at the best chunk and
 * chunk again at the best block; then, if base->tail_steps is 0, tail_steps in {4, 8, 16, 32, 64,
 * 128, 256, 512, never} for the best pair, and, if base->tail_cap is 0 too,
 * the pairs of tail_steps in {4, 8, 16, 32, 64} and tail_cap in {64, 128,
 * 256, no limit}, then, if base->pool_order is 0, each of the three pool orders,
 * then block and chunk once more at the final hand-off, cap and order (the
 * whole plane when calls take under 50 ms, else chunk, block, chunk).  Each candidate is timed with HIP
 * events on `stream` (median of `reps` launches after one untimed launch);
 * the eight fastest distinct launches are then timed again, round-robin,
 * 3 * reps + 1 launches each, and the lowest median wins (2 * reps + 2
 * untimed launches come first, so start-up clocks do not count).  Trials run on the
 * caller's boxes; the boxes' states are snapshotted first and restored
 * after every trial and at the end, so the caller's data is left unchanged.  The
 * winner is stored in the handle for the size bucket of these boxes (total
 * cells rounded to a power of two): later calls whose chunk_steps,
 * block_size, tail_steps or tail_cap are 0 use it.  If cache_path
 * is not NULL the result is also looked up in / written to that JSON file,
 * keyed by mechanism hash, size bucket and GPU architecture name; a cache hit
 * skips the sweep.  best (may be NULL) receives the chosen options.
 * Allocates the snapshots (and, on a miss, grows the workspace reservation to
 * the boxes' cells if it is smaller); synchronises `stream`.
 */
int chem_autotune(chem_mech m, const chem_box *boxes, int32_t n_boxes, const chem_opts *base,
                  int32_t reps, const char *cache_path, void *stream, chem_opts *best);

/* ------------------------------------------------------------------------
 * Learned surrogate.  The paper names machine-learned acceleration of the
 * chemistry as future work (Sec. 7) without a design; this one is an MLP
 * mapping one cell's (T, ln p, ln dt, Y_1..Y_N) to the increment
 * (dT, dY_1..dY_N) of one flow step: N+3 -> 128 -> 128 -> 128 -> N+1, SiLU
 * hidden layers, BF16 GEMM operands with FP32 accumulation on the matrix
 * cores, FP32 master weights, inputs and outputs standardised by the mean and
 * standard deviation of the first training set.  Parameter vector (FP32):
 * W1[128][N+3] b1[128] W2[128][128] b2 W3[128][128] b3 W4[N+1][128] b4[N+1];
 * normaliser vector (FP32): mu_in[N+3] sd_in[N+3] mu_out[N+1] sd_out[N+1]
 * zmin[N+3] zmax[N+3] (zmin/zmax: the standardised training hull).
 * ------------------------------------------------------------------------ */
typedef struct chem_surr_s *chem_surr; /* opaque, owned by the library */

/* Trust-test failure bits (0 = trusted). */
#define CHEM_TRUST_HULL 1      /* a standardised input outside [zmin - m, zmax + m] */
#define CHEM_TRUST_ELEM 2      /* an element mass fraction changed by more than elem_tol */
#define CHEM_TRUST_POS 4       /* some Y_k + dY_k < -pos_tol */
#define CHEM_TRUST_ENERGY 8    /* |e(T+dT, Y+dY) - e(T, Y)| / c_v(T, Y) > energy_tol [K] */
#define CHEM_TRUST_NONFINITE 16

/* New surrogate for mechanism m (hidden must be 128, depth 3); weights
 * He-uniform (bound sqrt(6/fan_in)) from a splitmix64 stream seeded by seed,
 * biases zero.  Synchronises the device. */
int surrogate_create(chem_mech m, int32_t hidden, int32_t depth, uint64_t seed, chem_surr *out);

/* Inputs N+3, outputs N+1 and parameter count of a surrogate. */
int surrogate_query(chem_surr s, int32_t *n_in, int32_t *n_out, int64_t *n_params);

/* Copy the FP32 parameter and normaliser vectors to / from host memory
 * (either pointer may be NULL).  Synchronise the device. */
int surrogate_get_params(chem_surr s, float *theta_host, float *norm_host);
int surrogate_set_params(chem_surr s, const float *theta_host, const float *norm_host);

/*
 * Training pairs from two SoA state blocks of the same cells (layout as
 * above): X[i] = (T, ln p, ln dt, Y_1..Y_N) of `before` (p from the ideal gas
 * law, dt = dt_cells[i] if dt_cells is not NULL, else dt) and
 * Y[i] = after - before for (T, Y_1..Y_N).  X is float[n][N+3], Y is
 * float[n][N+1], all device memory.  Enqueue only.
 */
int surrogate_make_pairs(chem_mech m, const double *before, const double *after, int64_t ld,
                         int64_t n, double dt, const double *dt_cells, float *X, float *Y,
                         void *stream);

/*
 * Train on n raw pairs (device float X[n][N+3], Y[n][N+1]): the first call
 * fits the normaliser and the hull on its data; then `epochs` passes of
 * floor(n / batch) Adam steps (beta 0.9 / 0.999, eps 1e-8, learning rate
 * lr with a cosine decay to zero over the call) on the MSE of the
 * standardised outputs.  Each epoch visits samples in the order
 * i -> (a i + b) mod n with a coprime to n, drawn from `seed`.  loss_host
 * (may be NULL) receives the mean training loss of each epoch.  Synchronises
 * `stream`.
 */
int surrogate_train(chem_surr s, const float *X, const float *Y, int64_t n, int32_t epochs,
                    int32_t batch, float lr, uint64_t seed, void *stream, float *loss_host);

/* Network outputs (standardised, float[n][N+1]) for raw inputs X
 * (float[n][N+3]).  Synchronises `stream`. */
int surrogate_forward(chem_surr s, const float *X, int64_t n, float *out, void *stream);

/* Gradient of the batch MSE for already standardised Xn[B][N+3], Yn[B][N+1]
 * into grad_out (device float[n_params], may be NULL); loss_host (may be
 * NULL) receives the loss and then the call synchronises `stream`. */
int surrogate_grad(chem_surr s, const float *Xn, const float *Yn, int32_t B, float *grad_out,
                   float *loss_host, void *stream);

/*
 * Allocate what surrogate_infer with fallback needs for up to max_cells
 * cells: the fallback list (4 B per cell; the fallback's integration uses
 * the mechanism's workspace).  Growing it
 * first waits for the whole device.  CHEM_EINVAL for a null handle or
 * max_cells < 0.
 */
int surrogate_reserve(chem_surr s, int64_t max_cells);

/*
 * One flow step of dt for n_cells cells through the surrogate: features in
 * FP64, the MLP on the matrix cores, then the FP64 trust test with
 * trust = {hull_margin, elem_tol, pos_tol, energy_tol}.  Trusted cells get
 * T + dT and max(Y + dY, 0) in place (rho and h untouched; the trust test
 * allows Y + dY down to -pos_tol, the write clips it to 0).  Untrusted cells keep their
 * state and, if `fallback` is non-zero, are integrated from it by the FP64
 * LSRK path (opts as for chem_integrate) in the same stream, with no host
 * round trip: the inference kernel appends the untrusted cells to a
 * device-side list that one pool of the persistent kernel then takes.
 * With fallback, a cell outside the training hull is decided by that
 * criterion alone (trust code CHEM_TRUST_HULL, the others not evaluated),
 * and a 64-cell tile holding only such cells skips the network.  Optional
 * device outputs: trust_code int32[n] (CHEM_TRUST_* bits), out_std
 * float[n][N+1] (raw network outputs; not written for a skipped tile),
 * status / counts (as chem_integrate,
 * written for fallback cells only).  n_fallback_host (may be NULL) receives
 * the number of untrusted cells and then the call synchronises `stream`.
 * Allocates nothing: with fallback, n_cells must be within both the
 * surrogate's reservation (surrogate_reserve) and the mechanism's
 * (chem_workspace_reserve), else CHEM_ECAPACITY.
 */
int surrogate_infer(chem_surr s, chem_mech m, double *state, int64_t ld, int64_t n_cells, double dt,
                    const double trust[4], int32_t fallback, const chem_opts *opts, void *stream,
                    int32_t *trust_code, float *out_std, int32_t *status, int32_t *counts,
                    int64_t *n_fallback_host);

/*
 * Tune the launch of surrogate_infer's FP64 fallback (block_size,
 * chunk_steps, tail_steps, tail_cap, pool_order of `opts`) for this state
 * block by the search of chem_autotune, each trial a whole
 * surrogate_infer(fallback = 1) call on the block as it is on entry (the
 * launch is chosen on the surrogate step itself: the fallback pool's cells
 * sit scattered in the block, in the order the list was built).  The
 * block is restored after every trial and on return.  `base` gives rtol,
 * atol, max_steps and the scheme, and any launch field it fixes.  A cache
 * entry (key hash:size-bucket:arch:surrogate, file as for chem_autotune)
 * is returned without tuning; otherwise the result is appended to it.  The
 * result goes to *best only (the mechanism's tuned table is for plain
 * integrations).  A set-up call: reserves what the trials need, allocates a
 * snapshot of the block and synchronises `stream`.  CHEM_EINVAL for null
 * arguments, n_cells <= 0 or ld < n_cells.
 */
int surrogate_autotune(chem_surr s, chem_mech m, double *state, int64_t ld, int64_t n_cells,
                       double dt, const double trust[4], const chem_opts *base, int32_t reps,
                       const char *cache_path, void *stream, chem_opts *best);

/*
 * Capture one surrogate step with fallback (surrogate_infer with
 * fallback = 1 on this block, dt, trust and opts; no trust codes, outputs,
 * status or counts) into a HIP graph launched with chem_graph_launch and
 * freed with chem_graph_destroy: the inference kernel, then the FP64 pool
 * over the device-side list, whose length the kernels read when they run
 * (no memset nodes, no host round trip).  The graph owns its fallback list
 * and its pool's counter, tail records and order, so its launches may
 * follow eager calls on the same handles on one stream; two launches of one
 * graph must not overlap.  It uses the surrogate's weights and the
 * mechanism's tables as they are when launched.  A set-up call: allocates
 * (about 148 B per cell for 9 species) and synchronises `stream` before
 * capturing on a private stream.  CHEM_EINVAL for null arguments,
 * n_cells <= 0 or ld < n_cells.
 */
int surrogate_graph_capture(chem_surr s, chem_mech m, double *state, int64_t ld, int64_t n_cells,
                            double dt, const double trust[4], const chem_opts *opts, void *stream,
                            chem_graph *out);

/* Save / load parameters and normaliser (binary; tied to the mechanism hash). */
int surrogate_save(chem_surr s, const char *path);
int surrogate_load(chem_mech m, const char *path, chem_surr *out);

/* Release a surrogate (synchronises the device). */
void surrogate_free(chem_surr s);

/* Message for a return code; valid for the life of the process. */
const char *chem_strerror(int code);

/* Message for the calling thread's most recent failure ("" if none). */
const char *chem_last_error(void);

/* Diagnostics: y[i] = e^x[i] for i < n (device arrays, caller-owned), with
 * the exponential the rate evaluation uses (Cody-Waite reduction and a
 * degree-11 Chebyshev polynomial; within 1 ulp of the correctly rounded value), so it
 * can be checked against a reference.  Enqueued on `stream`. */
int chem_eval_exp(const double *x, double *y, int64_t n, void *stream);

/* Diagnostics for every elementary function the integrators use in place of
 * the library's: y[i] = fn(x[i]) for i < n (device arrays, caller-owned),
 * enqueued on `stream`.  fn is one of
 *   CHEM_MATH_EXP_CW      the per-lane rate exponential (as chem_eval_exp);
 *   CHEM_MATH_LOG_ATANH   the logarithm of ln T (reduction to [sqrt(1/2),
 *                         sqrt(2)) and the atanh series; within 1 ulp for
 *                         finite x > 0, NaN otherwise);
 *   CHEM_MATH_EXP_TAB     the cooperative kernel's rate exponential (a table
 *                         of 2^(j/64) in LDS and a degree-6 polynomial;
 *                         about 1 ulp at most on [-745, 709]).
 * (1 is not used.)  CHEM_EINVAL for an unknown fn, n < 0 or a null array with
 * n > 0. */
#define CHEM_MATH_EXP_CW 0
#define CHEM_MATH_LOG_ATANH 2
#define CHEM_MATH_EXP_TAB 3
int chem_eval_math(int32_t fn, const double *x, double *y, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CHEMGPU_H */
