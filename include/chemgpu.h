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
#define CHEM_ECAPACITY (-6)    /* more cells than the reserved workspace holds */

/* Per-cell status codes written to the status array. */
#define CHEM_CELL_OK 0          /* reached dt */
#define CHEM_CELL_MAXSTEPS 1    /* step budget (accepted + rejected) exhausted before dt */
#define CHEM_CELL_NONFINITE 2   /* non-finite input; the cell was left unchanged */
#define CHEM_CELL_H_UNDERFLOW 3 /* step size fell below 1e-14 * dt */

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
 * bytes.  *out receives a handle to free with chem_mech_free. */
int chem_mech_load(const char *path, chem_mech *out);

/* Species count N, reaction count and content hash of a loaded mechanism. */
int chem_mech_query(chem_mech m, int32_t *n_species, int32_t *n_reactions, uint64_t *hash);

/* Release a mechanism and its workspace (destroy its graphs first). */
void chem_mech_free(chem_mech m);

/* Reserve the device workspace (work queue, per-cell progress) for up to
 * max_cells cells.  All device allocation of the integrate calls happens here
 * or, if never called, on the first integrate call that needs it. */
int chem_workspace_reserve(chem_mech m, int64_t max_cells);

/*
 * Advance n_cells cells by dt (paper Eq. 20-22), in place.
 *   status: NULL or int32[n_cells] device array of CHEM_CELL_* codes.
 *   counts: NULL or int32[2 * n_cells] device array; counts[i] = accepted
 *           steps, counts[n_cells + i] = rejected steps of cell i.
 * Enqueued on `stream`; no host synchronisation.
 */
int chem_integrate(chem_mech m, double *state, int64_t ld, int64_t n_cells, double dt,
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
 * table is copied to the device through a pinned staging buffer owned by the
 * mechanism handle; the call returns without waiting for the GPU.
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
 * Autotune block size and chunk length for these boxes: every candidate
 * (block in {64, 128, 192, 256, 384, 512} that fits the LDS compaction slots,
 * chunk in {1, 2, 4, 8, 16, 32, 64}) is timed with HIP events on `stream`
 * (median of `reps` launches) on the caller's boxes; the boxes' states are
 * snapshotted first and restored after every trial and at the end, so the
 * caller's data is left unchanged.  The winner is stored in the handle for
 * the size bucket of these boxes (total cells rounded to a power of two):
 * later calls whose chunk_steps and block_size are 0 use it.  If cache_path
 * is not NULL the result is also looked up in / written to that JSON file,
 * keyed by mechanism hash, size bucket and GPU architecture name; a cache hit
 * skips the sweep.  best (may be NULL) receives the chosen options.
 * Synchronises `stream`.
 */
int chem_autotune(chem_mech m, const chem_box *boxes, int32_t n_boxes, const chem_opts *base,
                  int32_t reps, const char *cache_path, void *stream, chem_opts *best);

/* Message for a return code; valid for the life of the process. */
const char *chem_strerror(int code);

/* Message for the calling thread's most recent failure ("" if none). */
const char *chem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CHEMGPU_H */
