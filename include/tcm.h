/*
 * tcm.h -- C-ABI of libtcm.so: the Triggered Cells Method (TCM) hot path on
 * one AMD Instinct MI355X (gfx950).
 *
 * Problem statement (Introduction, eq.(1)-(4)): the scalar wave equation
 * (1/c^2) d2phi/dt2 = lap(phi) on a grid with dx = dy = dz, advanced by the
 * second-order leapfrog of eq.(3)
 *
 *     phi^{n+1} = 2 phi^n - phi^{n-1} + (c dt / dx)^2 [sum of 6 neighbours - 6 phi^n]
 *
 * with the field zero outside the domain.  The TCM ("The Triggered Cells
 * Method", "Cells construction", "Boxes", "Updating active cells") splits the
 * grid into cells of 8^3 nodes ("blocks" below); only active blocks hold
 * memory (a slot of the device pool) and are updated.  A block is activated
 * when |phi^{n+1}| on the face of an active neighbour exceeds `trigger`, and
 * released when every |phi^{n+1}| and |phi^n| in it is at most `retire` and no
 * neighbour triggers it.  Source blocks stay active while their source has
 * samples left ("Source insertion").
 *
 * Arithmetic: FP32 fields; C2 = (float)(t * t) with t = (double)c * dt / dx;
 * per node, s = ((x+ + x-) + (y+ + y-)) + (z+ + z-), lap = s - 6 phi,
 * next = (2 phi - prev) + C2 lap, no fused multiply-add, subnormals kept.
 *
 * Conventions shared by every call:
 *  - Linear node index i = x + nx (y + ny z) (x fastest) for host arrays.
 *  - Time: phi^0 = phi^{-1} = 0 at creation; after k steps the current level
 *    is phi^k.  Sample j of a source added when the current level was phi^s
 *    is added to phi^{s+j+1} (the step that computes it).
 *  - Every call returns a tcm_status and never aborts; tcm_last_error() gives
 *    the message of the last failure on that handle.
 *  - Host input arrays are copied before the call returns.  Output buffers
 *    belong to the caller.  The handle owns all device memory it allocates; a
 *    caller-supplied device_pool must outlive the handle.
 *  - A handle is not thread-safe; distinct handles are independent.
 *  - Work is issued on the handle's stream.  Calls that return data to the
 *    host (tcm_read, tcm_read_traces, tcm_stats) synchronise that stream;
 *    tcm_step synchronises once at its end to report device errors.
 */
#ifndef TCM_H
#define TCM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tcm_handle tcm_handle;

typedef enum {
    TCM_OK = 0,
    TCM_E_ARG = -1,     /* invalid argument (c < 0 or not finite, thresholds, sizes) */
    TCM_E_CFL = -2,     /* eq.(4) violated: (cmax dt / dx)^2 * 3 > 1 (+4 ulp) */
    TCM_E_POOL = -3,    /* more active blocks than pool slots; sticky, see tcm_step */
    TCM_E_RANGE = -4,   /* source, receiver or read box outside the domain */
    TCM_E_DEVICE = -5,  /* HIP runtime error; the handle is poisoned (destroy only) */
    TCM_E_STATE = -6,   /* call not valid in the handle's state */
    TCM_E_NOMEM = -7,   /* device or host allocation failed */
    TCM_E_NONFINITE = -8 /* a field value became NaN or infinite; sticky, like TCM_E_POOL */
} tcm_status;

enum { TCM_MEDIA_DENSE = 0, TCM_MEDIA_LAYERED = 1, TCM_MEDIA_LATTICE = 2 };
enum { TCM_ENGINE_BLOCKS = 0, TCM_ENGINE_DENSE = 1 };
enum {
    TCM_FLAG_TIMING = 1,    /* time every block-stencil launch with HIP events */
    TCM_FLAG_NO_GRAPH = 2,  /* launch each step's kernels directly (no hipGraph replay) */
    TCM_FLAG_NO_UNIFORM_C2 = 4, /* always read the per-node C2 plane (no scalar C2 for
                                   blocks whose C2 is uniform, "Media" hybrid engine) */
    TCM_FLAG_THREE_PASS_UPDATE = 8, /* run the activation update as plan, allocation and
                                   compaction launches even where the two-launch update applies
                                   (constant levels, update every step, no shutdown, one pool
                                   slot per block key, at most 2^24 keys); the results are the same */
    TCM_FLAG_DEBUG_CHECKS = 16, /* tcm_step runs tcm_check at its end and returns TCM_E_STATE
                                   when a table invariant is violated */
    TCM_FLAG_C2_PLANES = 32     /* read every non-uniform block's C2 plane (by default, with
                                   constant levels and lattice media of spacing >= 8, a block
                                   inside the domain takes its C2 from the 8 corners of its
                                   lattice cell, computed as the media evaluation does, instead
                                   of reading its plane; TCM_FLAG_NO_UNIFORM_C2 implies this
                                   flag); the results are the same */
};

/* Run configuration.  Zero-initialise, then set the fields. */
typedef struct {
    int32_t  nx, ny, nz;      /* grid nodes (single shot; ignored by tcm_create_batch) */
    double   dx, dt;          /* node spacing (dx = dy = dz) and time step */
    float    trigger;         /* activation level on |phi^{n+1}| at a block face, >= 0 */
    float    retire;          /* keep level on |phi| inside a block, 0 <= retire <= trigger */
    uint64_t pool_bytes;      /* pool cap in bytes (6 KiB per slot); 0: one slot per block
                                 key (the blocks of the domain, padded to whole 4x4x4 tiles),
                                 limited to 90 % of free device memory */
    void*    device_pool;     /* optional caller device memory of >= pool_bytes (then
                                 pool_bytes is required, TCM_E_ARG otherwise); NULL: own */
    void*    stream;          /* hipStream_t to issue work on; NULL: a stream of the handle */
    int32_t  engine;          /* TCM_ENGINE_BLOCKS (the TCM) or TCM_ENGINE_DENSE (every node) */
    int32_t  flags;           /* TCM_FLAG_* */
    int32_t  checkpoint_every;/* > 0 keeps forward checkpoints every k steps for tcm_adjoint */
    int32_t  graph_steps;     /* steps per captured hipGraph (0: 16) */
    int32_t  wg_per_cu;       /* block-stencil workgroups per compute unit (0: default) */
    int32_t  shutdown_steps;  /* shutdown process, eq.(6): a block that no longer qualifies
                                 stays shutdown_steps more steps with both field levels
                                 multiplied by shutdown_alpha after each, then is released;
                                 0 releases at once.  At most 255. */
    float    shutdown_alpha;  /*   the decay factor alpha; total attenuation A = alpha^n */
    float    trigger_rel;     /* adaptive levels (Table 1 Trig_level): each step uses
                                 max(trigger, trigger_rel * M) and max(retire, retire_rel * M),
                                 M = max |phi^{n+1}| over the domain after insertion; */
    float    retire_rel;      /*   0 <= retire_rel <= trigger_rel; both 0: constant levels */
    int32_t  trigger_interval;/* activation update after every k-th step (eq.(5)), 1 <= k <= 8
                                 (0: 1).  With k > 1 a block holding any |phi| above the
                                 trigger activates all 26 nearest and diagonal blocks (Figure 3),
                                 and a source block's 26 neighbours are activated with it, so
                                 that trigger = retire = 0 stays equal to the dense grid. */
    int32_t  blocks_per_wg;   /* stencil workgroup tile: 2, 4 or 8 blocks taken as consecutive
                                 list entries, sharing x faces (0: 4) */
    int32_t  blocks_per_wave; /* 1: one block per wave; 2: each wave takes two consecutive
                                 entries of the tile and loads them together (tile of 4 or 8
                                 blocks); 0: 1 */
} tcm_config;

/* Wave-speed model ("Media": an array, or rules evaluated when a block is
 * allocated).  Values are in the same length/time units as dx and dt. */
typedef struct {
    int32_t       kind;           /* TCM_MEDIA_* */
    const float*  c;              /* DENSE: host array of nx*ny*nz speeds (x fastest) */
    int32_t       nlayers;        /* LAYERED: c = c_layer[k] for z_top[k] <= z < z_top[k+1] */
    const int32_t* z_top;         /*   ascending, z_top[0] == 0 */
    const float*  c_layer;
    const double* lattice;        /* LATTICE: lx*ly*lz FP64 node values (x fastest) on a lattice */
    int32_t       lx, ly, lz;     /*   of spacing 2^log2_spacing nodes; node (i,j,k) sits at */
    int32_t       log2_spacing;   /*   (i S, j S, k S); lx > (nx-1)/S + 1 etc.  The node value is
                                       the trilinear interpolation, evaluated in FP64 in the order
                                       x, then y, then z, rounded once to FP32. */
} tcm_media;

/* One shot of a batch: its grid and media (tcm_create_batch). */
typedef struct {
    int32_t   nx, ny, nz;
    tcm_media media;
} tcm_shot;

typedef struct {
    int64_t step;                 /* current level n (fields hold phi^n and phi^{n-1}) */
    int64_t active_blocks;        /* blocks updated by the next step */
    int64_t peak_active_blocks;
    int64_t pool_slots;           /* capacity of the pool */
    int64_t pool_bytes;           /* bytes of the pool (slots * 6 KiB) */
    int64_t peak_pool_bytes;      /* peak_active_blocks * 6 KiB */
    int64_t table_bytes;          /* other device memory: block table, bitmap, lists, media */
    int64_t activations;
    int64_t retirements;
    int64_t cell_updates;         /* in-domain nodes updated so far (dense: nodes x steps) */
    int32_t error;                /* sticky device error (TCM_E_POOL, TCM_E_NONFINITE) or 0 */
    int32_t nshots;
    double  stencil_ms;           /* TCM_FLAG_TIMING: summed block-stencil kernel time */
    int64_t stencil_launches;     /* TCM_FLAG_TIMING: launches summed in stencil_ms */
    int64_t stencil_cells;        /* TCM_FLAG_TIMING: in-domain nodes of the timed launches */
    int64_t uniform_cell_updates; /* of cell_updates, nodes of blocks read with a scalar C2 */
    int64_t stencil_cells_uniform;/* TCM_FLAG_TIMING: of stencil_cells, nodes with a scalar C2 */
    int64_t decay_block_steps;    /* block-steps of the shutdown decay (eq.(6)) */
    double  trigger_level;        /* levels used by the last step (adaptive or constant) */
    double  retire_level;
    int64_t grad_cells;           /* TCM_FLAG_TIMING: nodes whose gradient term mu (L u) the adjoint-field
                                     launches formed (adjoint block active, forward block active a
                                     step before) */
    double  adjoint_field_ms;     /* TCM_FLAG_TIMING: summed block-stencil time of the adjoint field
                                     (each launch also adds the step's gradient terms) */
    int64_t adjoint_field_launches;
    int64_t adjoint_field_cells;  /* nodes those adjoint-field steps updated */
    int64_t adjoint_field_cells_uniform; /* of those, nodes of blocks with a scalar C2 */
    double  recompute_ms;         /* TCM_FLAG_TIMING: summed block-stencil time of the forward steps that
                                     tcm_adjoint recomputed (they also store L u per node) */
    int64_t recompute_launches;
    int64_t recompute_cells;      /* nodes those recomputed steps updated */
    int64_t recompute_cells_uniform; /* of recompute_cells, nodes of blocks with a scalar C2 */
    int64_t checkpoint_bytes;     /* device bytes of the stored forward checkpoints (sparse: the
                                     active blocks' two phi levels and tables, ~4 KiB per block) */
    int64_t checkpoints;          /* forward checkpoints stored */
    int64_t adjoint_bytes;        /* device bytes the last tcm_adjoint held besides the checkpoints:
                                     L u store, key maps, gradient blocks, adjoint-field pool and tables */
    /* of the counts above, nodes of blocks whose C2 the stencil formed from a
       lattice record (TCM_FLAG_C2_PLANES unset; the rest of the non-uniform
       nodes read their C2 plane) */
    int64_t lattice_cell_updates;        /* of cell_updates */
    int64_t stencil_cells_lattice;       /* of stencil_cells */
    int64_t adjoint_field_cells_lattice; /* of adjoint_field_cells */
    int64_t recompute_cells_lattice;     /* of recompute_cells */
} tcm_stats_t;

/* Create a single-shot handle (eq.(3) on an nx*ny*nz grid, "Cells construction").
 * Validates eq.(4) with the largest speed of `media` (TCM_E_CFL), speeds
 * (c >= 0 and finite; TCM_E_ARG), thresholds (TCM_E_ARG).  On success *out
 * owns a zero field with no active block. */
tcm_status tcm_create(const tcm_config* cfg, const tcm_media* media, tcm_handle** out);

/* Create a handle that runs `nshots` independent grids over one shared pool
 * and one active list (dt, dx, thresholds and pool from cfg). */
tcm_status tcm_create_batch(const tcm_config* cfg, const tcm_shot* shots, int32_t nshots,
                            tcm_handle** out);

/* Point source ("Source insertion"): sample j of w (host, nsamples values) is
 * added to phi^{s+j+1} at node (ix,iy,iz) of shot 0, where phi^s is the level
 * when the call is made.  Its block is activated now and kept active while
 * samples remain.  TCM_E_RANGE outside the domain; TCM_E_POOL if no slot. */
tcm_status tcm_add_source(tcm_handle* h, int32_t ix, int32_t iy, int32_t iz,
                          const float* w, int32_t nsamples);
tcm_status tcm_add_source_shot(tcm_handle* h, int32_t shot, int32_t ix, int32_t iy, int32_t iz,
                               const float* w, int32_t nsamples);

/* Advance nsteps leapfrog steps (eq.(3)) with block activation and release
 * every step ("Updating active cells", "Time stepping").  Returns TCM_E_POOL if
 * a step needed more slots than the pool has, TCM_E_NONFINITE if a step
 * produced a NaN or infinite value (the stencil checks every value it
 * writes): that step's phi^{n+1} is kept (the level advances to n+1 with the
 * old active set) and later steps do nothing; reads and stats stay valid. */
tcm_status tcm_step(tcm_handle* h, int32_t nsteps);

/* Check the block tables between two steps (Table 1's Cell2box / Box2cell
 * bijection, the active list holding each active block once, its neighbour
 * rows, and the current-set bitmap of the two-launch update); *violations
 * receives the number of violations (0 for a consistent state).
 * Synchronous; allocates a scratch array of one int per slot.  TCM_E_STATE
 * for the dense engine. */
tcm_status tcm_check(tcm_handle* h, int64_t* violations);

/* Copy phi^n (which = 0) or phi^{n-1} (which = 1), the two field levels
 * that eq.(3) keeps, of the box [x0,x0+sx)x[y0,y0+sy)x[z0,z0+sz) of shot 0
 * into out (sx*sy*sz floats, x fastest), on the host (out_is_device = 0) or
 * the device (1, on the handle's stream).  Nodes of inactive blocks read 0:
 * a cell that is not boxed holds no field ("Boxes", "Updating active
 * cells": an unboxed cell's values are dropped).  Synchronous for host
 * output.  TCM_E_RANGE for a box outside the domain, TCM_E_ARG for which
 * not 0 or 1 or a NULL out. */
tcm_status tcm_read(tcm_handle* h, int32_t which, int32_t x0, int32_t y0, int32_t z0,
                    int32_t sx, int32_t sy, int32_t sz, float* out, int32_t out_is_device);
tcm_status tcm_read_shot(tcm_handle* h, int32_t shot, int32_t which, int32_t x0, int32_t y0,
                         int32_t z0, int32_t sx, int32_t sy, int32_t sz, float* out,
                         int32_t out_is_device);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * read as tcm_read_shot into host memory `out` (sx*sy*sz floats, x fastest),
 * staged through a static device array of the library (8 Mi floats = 32 MiB
 * per GPU, kept until the process ends) instead of a staging buffer the
 * handle allocates.  Calls no hipMalloc / hipFree.  Every call on one GPU
 * uses that GPU's one staging array: calls that overlap on one GPU (other
 * threads, other handles) race.  Synchronises the handle's stream.
 * TCM_E_ARG for a box of more than 8 Mi nodes or a NULL out; TCM_E_RANGE
 * outside the grid. */
tcm_status tcm_read_noalloc(tcm_handle* h, int32_t shot, int32_t which, int32_t x0, int32_t y0,
                            int32_t z0, int32_t sx, int32_t sy, int32_t sz, float* out);

/* Receivers: rec_xyz holds nrec (x,y,z) triples of shot 0 (rec_shot NULL) or
 * of shots rec_shot[r].  From the next step on, traces[k][r] = phi^{m+k+1} at
 * receiver r, where phi^m is the level when receivers were set. */
tcm_status tcm_set_receivers(tcm_handle* h, const int32_t* rec_xyz, const int32_t* rec_shot,
                             int32_t nrec);
/* Number of recorded steps (*nsteps) and the traces ([nsteps][nrec] floats). */
tcm_status tcm_read_traces(tcm_handle* h, float* out, int32_t out_is_device, int32_t* nsteps);

/* Gradient dJ/dc of a receiver misfit J with dJ/dtraces = resid ([nt][nrec],
 * host or device, rows for the first nt recorded steps) for the run made so
 * far from level 0 with checkpoint_every > 0.  The forward is recomputed
 * from checkpoints; the adjoint field mu = C2 lambda obeys the same update as
 * the forward, with sources C2_r resid.  grad_c: nx*ny*nz floats (shot 0).
 * TCM_E_STATE without checkpoints or if nt exceeds the recorded steps. */
tcm_status tcm_adjoint(tcm_handle* h, const float* resid, int32_t nt, int32_t resid_is_device,
                       float* grad_c, int32_t out_is_device);

/* Launch-shape choice of the block engine (tcm_autotune). */
typedef struct {
    int32_t wg_per_cu;            /* chosen block-stencil workgroups per compute unit */
    int32_t graph_steps;          /* chosen steps per captured hipGraph */
    double  ms_per_step;          /* probe time per step of the choice */
    int32_t ncand;                /* candidates timed */
    int32_t cand_wg_per_cu[32];
    int32_t cand_graph_steps[32];
    double  cand_ms_per_step[32];
    int32_t blocks_per_wg;        /* chosen workgroup tile (blocks per workgroup) */
    int32_t cand_blocks_per_wg[32];
    int32_t blocks_per_wave;      /* chosen blocks per wave (1 or 2) */
    int32_t cand_blocks_per_wave[32];
    int32_t nfam;                 /* tcm_autotune_run: tile families timed over the whole run */
    int32_t fam_blocks_per_wg[8]; /*   each family's best probe shape ... */
    int32_t fam_blocks_per_wave[8];
    int32_t fam_wg_per_cu[8];
    double  fam_run_ms[8];        /*   ... and its whole-run time (best of two) */
} tcm_tuning;

/* Time probe_steps steps from the current state for each candidate launch
 * shape (workgroup tile of 2, 4 or 8 blocks, one or two blocks per wave, x
 * workgroups per CU of the persistent stencil grid, then steps per graph),
 * restore the state after
 * each probe, and keep the fastest shape for later tcm_step calls.  The
 * block edge stays 8 (one 64-lane wave per block).  The field, statistics
 * and traces are unchanged on return.  TCM_E_STATE for the dense engine or
 * a failed run; out may be NULL. */
tcm_status tcm_autotune(tcm_handle* h, int32_t probe_steps, tcm_tuning* out);

/* Pick the launch shape for a run of nsteps steps from the current state:
 * every candidate of tcm_autotune is probed for probe_steps steps at three
 * states along the run (a quarter, half and three quarters of the way,
 * reached with the current shape) and ranked by its mean probe time; the
 * steps per graph are chosen on the fastest; the best shape of each tile
 * family (blocks per workgroup x blocks per wave) then runs the whole run
 * from the current state twice, and the family with the fastest run is
 * kept (out->ms_per_step = its run time / nsteps; out->fam_* lists the
 * families' whole-run times).  The field, statistics and traces are
 * unchanged on return.  nsteps >= 4; TCM_E_STATE for the dense engine or a
 * failed run (also when the run fails while the tuner steps it). */
tcm_status tcm_autotune_run(tcm_handle* h, int32_t nsteps, int32_t probe_steps, tcm_tuning* out);

/* Set the launch shape directly (for example a stored tcm_autotune choice):
 * blocks_per_wg 2, 4 or 8 and blocks_per_wave 1 or 2 (2 needs a tile of 4
 * or 8; 0: keep either), wg_per_cu in [1, resident workgroups per CU for
 * that shape], graph_steps >= 1.  Block engine only; TCM_E_ARG out of
 * range. */
tcm_status tcm_set_launch(tcm_handle* h, int32_t wg_per_cu, int32_t graph_steps,
                          int32_t blocks_per_wg, int32_t blocks_per_wave);

/* Return to level 0 (zero field, no active block, no sources, no traces);
 * media, configuration and allocations are kept. */
tcm_status tcm_reset(tcm_handle* h);

/* Replace the wave speed of one shot ("Media": an array or rules) by media
 * of the same kind and sizes as at creation (dense: nx*ny*nz speeds; layered:
 * the same layer count; lattice: the same lattice size and spacing), then
 * return the handle to level 0 as tcm_reset does (sources, receivers,
 * traces and checkpoints cleared).  The C2 planes follow the new speeds.
 * Lets a caller that runs many models of one geometry (an inversion) keep
 * one handle and its allocations.  Host data is copied before return.
 * TCM_E_ARG for another kind or size or invalid speeds, TCM_E_CFL if the
 * new speeds violate eq.(4) (the handle keeps its media then), TCM_E_RANGE
 * for a shot index out of range.  Snapshots taken before the call are
 * refused by tcm_restore (TCM_E_STATE). */
tcm_status tcm_set_media(tcm_handle* h, int32_t shot, const tcm_media* media);

/* Save the whole state at the current step (block engine: pool, block
 * tables and counters; dense engine: both field arrays) into device memory
 * that the snapshot owns; *snap receives an opaque pointer, freed by
 * tcm_snapshot_free.  The handle keeps its state.  TCM_E_NOMEM when the
 * device memory is short. */
tcm_status tcm_snapshot(tcm_handle* h, void** snap);

/* Return h to the step and state of a snapshot of h.  Stepping on from
 * there repeats the same results.  TCM_E_ARG for a snapshot of another
 * handle; TCM_E_STATE when sources or receivers were added since the
 * snapshot (they are part of the state: a source boxes its block when it is
 * added). */
tcm_status tcm_restore(tcm_handle* h, const void* snap);

/* Free a snapshot (NULL is allowed).  Call before destroying its handle. */
void tcm_snapshot_free(void* snap);

tcm_status tcm_stats(tcm_handle* h, tcm_stats_t* out);

void tcm_destroy(tcm_handle* h);

/* Measurement helper, not part of the method: the HBM bandwidth that a
 * streaming kernel of the block stencil's shape reaches on the current
 * device, the ceiling its roofline fraction is compared with.  The kernel
 * computes dst[i] = src[i] (+ src[n + i] (+ src[2n + i])) for i < n in the
 * fastest streaming shape measured (two floats per lane, 512-byte wave
 * accesses, 16 KiB of each stream per workgroup pass, non-temporal loads and
 * stores); with nread = 3 it reads 12 and writes 4 bytes per element, the
 * stencil's mix.
 *   src      device, nread * n floats (the sources back to back), 8-byte aligned
 *   dst      device, n floats, 8-byte aligned; must not overlap src
 *   n        floats per source, > 0 and a multiple of 4096
 *   nread    1, 2 or 3
 *   wg_per_cu  workgroups (256 threads) per compute unit; 0 => 8
 *   reps     launches, 1..1000
 *   stream   hipStream_t, NULL => the null stream
 *   best_ms  host; the shortest launch, timed with events stamped at the
 *            dispatch's start and end
 * Synchronous.  The caller owns the buffers.  TCM_E_ARG for a bad argument
 * (message in tcm_last_error(NULL)); TCM_E_DEVICE for a HIP error. */
tcm_status tcm_hbm_probe(const float* src, float* dst, uint64_t n, int32_t nread, int32_t wg_per_cu,
                         int32_t reps, void* stream, float* best_ms);

/* Message of the last failed call on h, or of the last failed call without
 * a handle (create, probe) on this thread when h is NULL.  Never NULL. */
const char* tcm_last_error(const tcm_handle* h);

/* Library version string. */
const char* tcm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TCM_H */
