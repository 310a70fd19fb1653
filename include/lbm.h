/* lbm.h - C ABI of the MI355X two-component pseudopotential LBM library.
 *
 * The library advances the improved multicomponent pseudopotential lattice
 * Boltzmann model of Sedahmed, Coelho & Warda (arXiv:2111.08666): two
 * immiscible components with Shan-Chen cohesion (Sec. 2.1, Eq. 13, psi =
 * rho), IVSD fluid-solid adhesion (Sec. 2.2, Eqs. 15-17), a forced collision
 * with a density-weighted mixture relaxation time (Eqs. 1-11; SRT, or MRT /
 * TRT variants with the same viscosity law), pull streaming with half-way
 * bounce-back, and the pressure inlet/outlet treatment Set-3 (Sec. 2.3,
 * Eqs. 18-28).  Every step runs in HIP kernels on one GPU.
 *
 * Conventions shared by every entry point:
 *  - Host pointers are read during the call only; nothing is retained.
 *  - Device memory is owned by the caller: the workspace handed to
 *    lbm_create / lbm_batch_create is borrowed until the matching destroy.
 *    The library itself allocates no device memory.
 *  - All GPU work is enqueued on the caller's HIP stream (hipStream_t passed
 *    as void*; NULL = the default stream), in stream order.  Only
 *    lbm_observables, lbm_get_density with a host destination, lbm_save,
 *    lbm_load, lbm_set_bc, the autotune calls and the create calls
 *    synchronise that stream.
 *  - Every call returns an lbm_status; on failure lbm_last_error() returns a
 *    message.  Invalid arguments are rejected before any device work.
 *  - A context is not thread-safe; distinct contexts are independent.
 *  - Fields are indexed with x fastest: node (x, y, z) is at
 *    x + nx * (y + ny * z).  Component 1 (index 0) is the invading,
 *    non-wetting fluid driven in at x = 0; component 2 (index 1) is the
 *    resident, wetting fluid held at x = nx - 1.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* bad argument; nothing was done */
  LBM_ENOMEM = -2,    /* workspace too small or misaligned */
  LBM_EDEVICE = -3,   /* a HIP call failed */
  LBM_EUNSTABLE = -4, /* a density became non-finite */
  LBM_ESTATE = -5     /* call not valid in the current state */
} lbm_status;

enum { LBM_SRT = 0, LBM_MRT = 1, LBM_TRT = 2 };            /* lbm_params.collision */
enum { LBM_STORE_F32 = 0, LBM_STORE_BF16DEV = 1 };          /* lbm_params.storage */
enum { LBM_MATH_F32 = 0, LBM_MATH_F64 = 1 };                /* lbm_params.math */
enum { LBM_AUTO = 0, LBM_FUSED = 1, LBM_SPLIT = 2, LBM_COMPACT = 3,
       LBM_FUSED_LIST = 4, LBM_COMPACT_FUSED = 5 };         /* lbm_params.strategy */

/* Problem geometry (Sec. 2.3 and Sec. 4.2: a solid map phi, periodic or
 * open axes, the inlet at x = 0 and the outlet at x = nx - 1). */
typedef struct {
  int32_t q;              /* 9 (D2Q9) or 19 (D3Q19) */
  int32_t nx, ny, nz;     /* nz = 1 for D2Q9 */
  const uint8_t *solid;   /* host, nx*ny*nz bytes, 1 = solid (phi of Eq. 16) */
  uint32_t periodic;      /* bit0 x, bit1 y, bit2 z */
  int32_t open_x;         /* 1: pressure inlet x = 0 and outlet x = nx-1 */
  int32_t porous_x0;      /* saturation window [porous_x0, porous_x1) */
  int32_t porous_x1;      /* 0 = nx */
} lbm_geometry;

/* Model parameters (Sec. 2 and Sec. 3). */
typedef struct {
  double tau[2];          /* tau^(1), tau^(2) > 1/2; nu = (tau - 1/2)/3 */
  double G;               /* G_coh = G_ads (Eq. 13, Sec. 2.2) */
  double xi;              /* wettability: chi1 = 1 + xi, chi2 = 1 - xi, |xi| < 1 */
  double rho_in1;         /* component-1 density at the inlet (Eqs. 22-25) */
  double rho_out2;        /* component-2 density at the outlet (Eqs. 18-21) */
  double rho_in2;         /* Set-1 only: component-2 inlet density */
  double rho_out1;        /* Set-1 only: component-1 outlet density */
  double g[3];            /* body acceleration, F^b = rho^s g (Eq. 12) */
  int32_t collision;      /* LBM_SRT (Eq. 1), LBM_MRT, LBM_TRT */
  int32_t bc_set;         /* 3 = Set-3 (the paper's); 1, 2 = Set-1, Set-2 */
  int32_t half_force_shift; /* 1: u = (j + F/2)/rho (default); 0: u = j/rho */
  int32_t mrt_sj_mode;    /* MRT component-momentum rate s_j: 0 = min(s_nu, s_q)
                             (default; stable from viscosity ratio 1 to 100),
                             1 = s_q, 2 = s_nu */
  double lambda;          /* magic (1/s_nu - 1/2)(1/s_q - 1/2); <= 0: s_q = s_nu */
  double s_e, s_eps;      /* MRT energy-mode rates; <= 0: equal to s_nu */
  int32_t storage;        /* LBM_STORE_F32 or LBM_STORE_BF16DEV: how f* is held */
  int32_t math;           /* node arithmetic: LBM_MATH_F32 (default: the
                             collision works on departures from w_i rho with
                             FP64 density sums, and stays within 1e-5 of
                             FP64 over 200 steps) or LBM_MATH_F64 */
  int32_t strategy;       /* LBM_AUTO, LBM_FUSED (one launch per step, halo
                             densities recomputed per block), LBM_SPLIT
                             (density, solid-density and collide launches) or
                             LBM_COMPACT (the split step over a compacted
                             layout that stores fluid nodes only: thread per
                             fluid node, bounce-back from the node's own
                             slots); LBM_FUSED_LIST (D2Q9: the fused
                             step whose collision phase runs over a per-tile
                             list of fluid nodes, their pulled populations
                             parked in LDS; nx up to about 1.8 million);
                             LBM_COMPACT_FUSED (the fused step over the
                             compacted layout of LBM_COMPACT: D2Q9, the
                             fused tile step; D3Q19 with FP32 storage, a
                             tile march that pulls every population once and
                             sums the next step's densities on chip, which
                             the context then carries between steps, plus a
                             pull for the tiles' edge nodes and the solid
                             densities of Eq. 17: three launches).
                             The layout is fixed at creation: the compacted
                             strategies cannot be switched to or from the
                             others (lbm_autotune stays within the layout).
                             LBM_AUTO: D3Q19 compacted; D2Q9 dense fused
                             while the two population buffers of all
                             instances of the context or batch fit in the
                             256 MB last-level cache, else compacted fused
                             (every instance must then be LBM_AUTO). */
  int32_t tile_rows;      /* fused D2Q9 tile height: 8, 12 or 16 (0 = 12);
                             for the compacted layouts in 3D, the rows per
                             band of the fluid-node numbering (bands of rows,
                             z-slice by z-slice; 0 = sized from the grid) */
  int32_t eq26_mode;      /* reading of Eqs. 26-27 (the outlet links of component 1
                             in Set-2 and Set-3, the inlet links of component 2 in
                             Set-2), which the paper says maintain themselves
                             through collision and streaming: 0 (default) they
                             keep their initial values; 1 they take the node's
                             own post-collision values, the rule of Eq. 28 */
  int32_t ivsd_frozen;    /* reading of Eq. 17, which the paper also evaluates at
                             t = 0: 0 (default) the virtual solid density follows
                             the current fluid densities every step; 1 it is
                             evaluated once, on the initial densities (those of
                             lbm_create or lbm_init_from_saturation), and held
                             (checkpoints carry the held values) */
} lbm_params;

/* Observables at the current time (Eq. 14 pressure, Sec. 4.2 saturation).
 * Sums are accumulated in FP64 on the GPU in a fixed order. */
typedef struct {
  int64_t step;
  double mass[2];         /* sum of rho^s over fluid nodes */
  double n_fluid;
  double n_window;        /* fluid nodes with porous_x0 <= x < porous_x1 */
  double sw_count;        /* window nodes with rho2 > rho1 */
  double sum_rho_w;       /* window sum of rho2 */
  double sum_rho;         /* window sum of rho1 + rho2 */
  double s_w;             /* sw_count / n_window */
  double s_w_weighted;    /* sum_rho_w / sum_rho */
  double p_in, p_out;     /* mean P = (rho1+rho2)/3 + G rho1 rho2 / 3 over face
                             nodes at least 3 nodes from any solid */
  double pc;              /* p_in - p_out */
  double n_in, n_out;
  int32_t flags;          /* bit0 non-finite density; bit1 a negative density (reported only:
                             a slightly negative minor-phase density near strongly
                             wetting walls is an artefact of the model, not a blow-up) */
  int32_t reserved;
  double stag[3];         /* staggered momentum per axis: the sum over fluid nodes of
                             (-1)^x j_x (resp. (-1)^y j_y, (-1)^z j_z), j the momentum of
                             both components' streamed populations, over the total
                             mass.  A checkerboard velocity mode that the densities do
                             not show; in long runs it can grow until a node diverges
                             (0 in 2D for z) */
} lbm_obs;

typedef struct lbm_ctx lbm_ctx;
typedef struct lbm_batch lbm_batch;

/* Size in bytes of the device workspace lbm_create needs (0 if invalid).
 * It depends on the layout the strategy implies (dense, or compacted to the
 * fluid nodes; see LBM_AUTO), so pass the same params to lbm_create. */
size_t lbm_workspace_bytes(const lbm_geometry *geom, const lbm_params *params);

/* Create a solver.  rho_init: host, 2*nx*ny*nz doubles (component 1 then 2;
 * values at solid nodes ignored) placed as rest equilibria w_i rho (the
 * first step starts by streaming them).  workspace: device, >= the size
 * above, 256-byte aligned.  Validates all inputs first (tau > 1/2, |xi| < 1,
 * finite non-negative densities, fluid nodes never touching a closed domain
 * edge, open-face fluid nodes with a fluid neighbour); then uploads the
 * geometry tables and initial state and synchronises the stream. */
lbm_status lbm_create(const lbm_geometry *geom, const lbm_params *params,
                      const double *rho_init, void *workspace, size_t ws_bytes,
                      void *hip_stream, lbm_ctx **out);

/* Change the Zou-He densities rho_in of component 1 at x = 0 and rho_out
 * of component 2 at x = nx - 1 (Eqs. 22-25 and 18-21; a pressure increment
 * of Sec. 4.2).  Both must be finite and > 0.  Takes effect from the next
 * step, captured graphs included; synchronises the stream. */
lbm_status lbm_set_bc(lbm_ctx *ctx, double rho_in1, double rho_out2);

/* Enqueue n time steps of Sec. 2 (streaming with bounce-back, Set-3 faces,
 * densities, solid densities of Eq. 17, forces of Eq. 13, collision of
 * Eqs. 1-11): one kernel launch per step for the fused strategies, three for
 * the split and compacted ones.  Asynchronous.  LBM_EUNSTABLE once
 * lbm_observables has seen a non-finite density. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* Capture n steps into a HIP graph once (again when n changes) and replay
 * it `reps` times; for launch-bound small domains.  n must be even; the
 * stream must not be the default stream (LBM_ESTATE).  Asynchronous. */
lbm_status lbm_step_graph(lbm_ctx *ctx, int64_t n, int64_t reps);

/* Observables at the current time; synchronises the stream.  Returns
 * LBM_EUNSTABLE (with *out filled) once a density is non-finite (flags bit0);
 * later lbm_step calls then return LBM_EUNSTABLE too. */
lbm_status lbm_observables(lbm_ctx *ctx, lbm_obs *out);

/* Densities rho^s at the current time as float, 2*nx*ny*nz values
 * (component 1 then 2; 0 at solid nodes).  dst_is_device = 1: dst is a
 * device pointer (stream-ordered); 0: host pointer (synchronises). */
lbm_status lbm_get_density(lbm_ctx *ctx, float *dst, int32_t dst_is_device);

/* Warm start from a saturation field (a learned surrogate's prediction of
 * the steady state, Sec. 4.2 drainage): replace the state by the rest
 * equilibria w_i rho of densities set node by node, (rho1, rho2) =
 * (rho_major, rho_minor) where sat > threshold (component 1, the invading
 * non-wetting fluid, fills the node) and (rho_minor, rho_major) elsewhere,
 * at every fluid node.  sat: nx*ny*nz floats, x fastest, values at solid
 * nodes ignored; a device pointer (sat_is_device = 1, stream-ordered) or a
 * host pointer (0: copied through the workspace; synchronises).  The held
 * boundary links of Eqs. 26-27 keep their values and the step counter
 * restarts at 0.  The densities must be finite and >= 0 with a positive
 * sum (LBM_EINVAL). */
lbm_status lbm_init_from_saturation(lbm_ctx *ctx, const float *sat, int32_t sat_is_device, double threshold,
                                    double rho_major, double rho_minor);

/* Debug aid for tests of failure handling (it computes nothing of the
 * paper): overwrite one stored value of fluid node (x, y, z) in the current
 * state, the post-collision populations the next step streams.  FP32
 * storage: population f*_i of component s (0 or 1), i in [0, q).  BF16-
 * deviation storage: the node's FP32 density word of component s, from
 * which every population of that node and component is rebuilt (i is
 * checked but not used).  A NaN makes the next observables report
 * LBM_EUNSTABLE without any device fault.  LBM_EINVAL for a NULL handle, a
 * node outside the grid or solid, or s or i out of range.  Synchronises
 * the stream. */
lbm_status lbm_debug_poke(lbm_ctx *ctx, int32_t x, int32_t y, int32_t z, int32_t s, int32_t i, float value);

/* Checkpoint: all state needed to continue bit-identically.  With
 * host_blob = NULL, *bytes receives the size.  Both synchronise. */
lbm_status lbm_save(lbm_ctx *ctx, void *host_blob, size_t *bytes);
lbm_status lbm_load(lbm_ctx *ctx, const void *host_blob, size_t bytes);

/* Steps taken since creation (as restored by lbm_load); -1 for NULL. */
int64_t lbm_get_step(const lbm_ctx *ctx);
/* Free the context (host memory only; the workspace stays the caller's).
 * Call it after the stream's pending work is done or abandoned. */
lbm_status lbm_destroy(lbm_ctx *ctx);

/* Last error message of ctx (or of the calling thread's last failed create
 * when ctx is NULL).  Never NULL. */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Name, grid size (blocks) and block size of the step kernel the context
 * launches (the collide kernel for the split and compacted strategies); for
 * profiling. */
lbm_status lbm_kernel_info(const lbm_ctx *ctx, char *name, size_t name_len,
                           int64_t *grid_blocks, int32_t *block_threads);

/* Time every step variant the context's layout allows (dense: fused and
 * listed at each tile height, split; compacted: the compacted step, and in
 * 2D the compacted fused step at each tile height) for `steps` steps each
 * (even, >= 2) with HIP events, in two passes over the variants (the better
 * time of each counts), and keep the fastest.  Every trial is 2 untimed and
 * `steps` timed ordinary steps: the state advances by
 * 2 x (number of variants) x (steps + 2).  report (optional) receives one
 * line per variant with its milliseconds per step.  Synchronises the stream. */
lbm_status lbm_autotune(lbm_ctx *ctx, int64_t steps, char *report, size_t report_len);

/* ---- batches: many instances of uneven size advanced together ----------
 * One launch per step covers every instance through a flat table of
 * (instance, tile) blocks; steps can be captured in one HIP graph.  All
 * instances must share q, storage, collision, math and layout (with
 * LBM_AUTO the batch's total decides the layout).  rho_inits[k] as for
 * lbm_create; each instance has its own geometry, parameters and
 * observables.  The calls mirror the single-context ones. */
size_t lbm_batch_workspace_bytes(int32_t k, const lbm_geometry *geoms, const lbm_params *params);
lbm_status lbm_batch_create(int32_t k, const lbm_geometry *geoms, const lbm_params *params,
                            const double *const *rho_inits, void *workspace,
                            size_t ws_bytes, void *hip_stream, lbm_batch **out);
lbm_status lbm_batch_step(lbm_batch *b, int64_t n);
/* n steps captured once into a HIP graph, replayed reps times (n even). */
lbm_status lbm_batch_step_graph(lbm_batch *b, int64_t n, int64_t reps);
lbm_status lbm_batch_observables(lbm_batch *b, lbm_obs *out /* k entries */);
/* Retire (active[i] == 0) or re-admit (non-zero) instances: host array of k
 * flags, all set at creation.  A retired instance is not advanced by
 * lbm_batch_step / lbm_batch_step_graph (the flat block table and the
 * per-instance launches leave it out, so it costs nothing); its state, step
 * count (lbm_obs.step) and density read-outs stay as they were, and a
 * re-admitted instance resumes from there bitwise as if it had never been
 * retired.  Active instances advance bitwise as in a batch without the
 * retired ones.  (LBM_COMPACT_FUSED in 3D rebuilds the psi it carries
 * between steps after a change, as after any change of state outside a
 * step; that rounds differently in the last FP32 place.)  A non-finite density in a retired instance does not stop
 * the batch (lbm_batch_observables still reports it in its flags).  A change
 * rebuilds the block table (synchronises the stream) and drops the captured
 * graph; no change is a no-op. */
lbm_status lbm_batch_set_active(lbm_batch *b, const int32_t *active);
lbm_status lbm_batch_get_density(lbm_batch *b, int32_t k, float *dst, int32_t dst_is_device);
lbm_status lbm_batch_destroy(lbm_batch *b);
const char *lbm_batch_last_error(const lbm_batch *b);
/* lbm_kernel_info and lbm_autotune for a batch: one variant is chosen for
 * the whole batch (every instance advances by variants x steps).  With the
 * split and compacted strategies each instance is launched on its own;
 * grid_blocks is then the largest instance's grid. */
lbm_status lbm_batch_kernel_info(const lbm_batch *b, char *name, size_t name_len,
                                 int64_t *grid_blocks, int32_t *block_threads);
lbm_status lbm_batch_autotune(lbm_batch *b, int64_t steps, char *report, size_t report_len);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
