/*
 * pbit.h — C ABI of the MI355X p-bit Ising-machine sweep library (libpbit.so).
 *
 * The library runs the simulated probabilistic-computing sweep of
 * "Probabilistic Computing Optimization of Complex Spin-Glass Topologies"
 * (arXiv 2510.23419) on one gfx950 GPU:
 *
 *   - the problem is a quadratic Ising Hamiltonian over N +-1 spins with
 *     symmetric couplings J (Sec. 1.1.1, Eq. 1), read here as
 *         E(m) = - sum_{bonds (i,j)} J_ij m_i m_j - sum_i h_i m_i ;
 *   - a p-bit sees the local field I_i = sum_j J_ij m_j + h_i (Sec. 1.2.1,
 *     Eq. 3) and resets to m_i = sgn(tanh(beta I_i) - u), u uniform on (-1, 1)
 *     (Sec. 1.2.1, Eq. 2, read with tanh and the annealing beta of Sec. 1.3.1);
 *   - spins of one update group (colour class) are updated together
 *     (Sec. 1.2.2); a sweep visits colour 0 then colour 1;
 *   - beta follows a caller-given schedule, one value per sweep (Sec. 1.3.1),
 *     over many independent replicas (Sec. 1.3.3).
 *
 * Three problem kinds are supported:
 *   PBIT_EA3D      periodic 3D Edwards-Anderson cube (Sec. 2), checkerboard
 *                  colouring (x + y + z) mod 2; every side even and >= 2;
 *   PBIT_BICLIQUE  complete bipartite K_{na,nb} (Sec. 3), side A colour 0;
 *   PBIT_GRAPH     any sparse graph given as a bond list, with k update groups
 *                  from a caller colouring or the greedy colouring of Sec. 1.2.2
 *                  (odd cubes and general QUBOs, Sec. 4.2); a sweep visits the
 *                  colour classes in ascending order.
 *
 * Determinism.  Every result is a pure function of (problem, beta schedule,
 * sweep range, replica range, seed, initial spins).  Randomness is
 * Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter (spin id,
 * absolute sweep index, global replica >> 2, domain); word (global replica & 3)
 * of the block belongs to the replica.  Domain 0 draws the updates; domain 1
 * (sweep 0) draws random initial spins: +1 if the word is below 2^31, else -1.
 * The decision uses the uint32 minority threshold
 *     Tm(beta, a) = ceil(ldexp(1 / (1 + exp((2 beta) a)), 32) - 0.5),  a = |I|,
 * evaluated in IEEE binary64 on the host; with s = sign(I) (+1 for I >= 0)
 * and x = ~w if I >= 0 else w, the new spin is -s if x < Tm and s otherwise.
 * Hence results do not depend on launch shapes, tile sizes or batching.
 *
 * Layouts at this boundary.
 *   EA site id      i = x + Lx * (y + Ly * z)
 *   EA couplings    int8 J[3][N]: J[d][i] is the bond (i, i + e_d), periodic
 *                   (d = 0, 1, 2 for x, y, z); with a side of 2 the two bonds
 *                   between a pair are distinct
 *   biclique sites  side A: 0..na-1, side B: na..na+nb-1
 *   biclique J      int8 J[na][nb] row-major, J[a][b] joins a and na + b
 *   fields          int8 h[N] or NULL (all zero)
 *   spins           int8 +-1, [replica][site]
 *   couplings must be in {-1, 0, +1} and fields in {-1, 0, +1}.
 *
 * Errors.  Every entry point returns PBIT_OK (0), PBIT_PENDING (1, poll
 * only) or a negative PBIT_E_* code, and never throws.  A failing call leaves
 * caller buffers and library state as they were, except PBIT_E_DEVICE, which
 * poisons the context (every later call on it returns PBIT_E_DEVICE).
 * pbit_last_error() returns a message for the calling thread's last failure.
 *
 * Ownership.  Input pointers are borrowed for the duration of the call; the
 * library copies what it keeps.  Output buffers are caller-allocated.
 * Problems and jobs belong to their context until unloaded / polled to
 * completion or until pbit_destroy.  A context may be used from several
 * threads; calls are serialised internally.
 */
#ifndef PBIT_H
#define PBIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PBIT_OK = 0,
    PBIT_PENDING = 1,
    PBIT_E_ARG = -1,         /* bad pointer, size, kind or option */
    PBIT_E_COLOURING = -2,   /* odd EA side or improper colouring */
    PBIT_E_RANGE = -3,       /* J or h outside {-1,0,1}, beta negative / NaN / inf */
    PBIT_E_NOMEM = -4,       /* the context's HBM budget (or the device) is exhausted */
    PBIT_E_BUSY = -5,        /* the serving queue is full */
    PBIT_E_HANDLE = -6,      /* unknown, stale or foreign problem / job handle */
    PBIT_E_DEVICE = -7,      /* HIP error; the context is poisoned */
    PBIT_E_UNSUPPORTED = -8  /* valid request the library does not handle (e.g. a general graph in a batch) */
};

enum { PBIT_EA3D = 1, PBIT_BICLIQUE = 2, PBIT_GRAPH = 3 };

typedef struct pbit_ctx pbit_ctx;

/* Create a context on HIP device `device`.  `hbm_budget_bytes` caps the device
 * memory the context may hold at once (problems, spins, tables, scratch);
 * 0 means "no cap beyond the device".  Writes the context to *out. */
int pbit_create(pbit_ctx **out, int device, uint64_t hbm_budget_bytes);

/* Destroy a context, its problems and pending jobs.  NULL is ignored. */
void pbit_destroy(pbit_ctx *ctx);

/* Message for the calling thread's last failing call ("" if none). */
const char *pbit_last_error(void);

/* Device memory currently held by the context, in bytes. */
uint64_t pbit_bytes_in_use(const pbit_ctx *ctx);

/* ---- problems (Sec. 1.1.1 Eq. 1; Sec. 2; Sec. 3) ------------------------ */

typedef struct {
    int32_t kind;           /* PBIT_EA3D or PBIT_BICLIQUE */
    int32_t dims[3];        /* EA: Lx, Ly, Lz (even, >= 2).  BICLIQUE: na, nb (>= 1), dims[2] ignored */
    const int8_t *J;        /* EA: [3][N].  BICLIQUE: [na][nb] */
    const int8_t *h;        /* [N] or NULL */
} pbit_problem_desc;

/* Validate and upload a problem; writes an opaque handle to *problem_out.
 * Errors: E_ARG, E_COLOURING (odd or zero EA side), E_RANGE, E_NOMEM, E_DEVICE. */
int pbit_load_problem(pbit_ctx *ctx, const pbit_problem_desc *desc, uint64_t *problem_out);

/* A general sparse graph (Sec. 1.2.2, Sec. 4.2).  Bond b joins bond_i[b] and
 * bond_j[b] (distinct, in [0, n_spins)) with coupling bond_J[b]; several bonds
 * may join the same pair and then add up.  colour[n_spins] (values below
 * n_colours) must be a proper colouring, or NULL for the greedy colouring:
 * vertices in ascending order each take the smallest colour none of their
 * already coloured neighbours has (at most max degree + 1 colours).  Every
 * vertex may have at most 127 bonds (E_UNSUPPORTED otherwise). */
typedef struct {
    int32_t n_spins;
    int32_t n_bonds;
    const int32_t *bond_i;
    const int32_t *bond_j;
    const int8_t *bond_J;   /* in {-1, 0, +1} */
    const int8_t *h;        /* [n_spins] or NULL */
    const uint8_t *colour;  /* [n_spins] or NULL */
    int32_t n_colours;      /* with colour: number of classes (1..255) */
} pbit_graph_desc;

/* Validate and upload a general graph; errors as pbit_load_problem. */
int pbit_load_graph(pbit_ctx *ctx, const pbit_graph_desc *desc, uint64_t *problem_out);

/* The colouring a problem's sweep uses: colour_out[N] (or NULL) and the
 * number of colour classes. */
int pbit_problem_colouring(pbit_ctx *ctx, uint64_t problem, uint8_t *colour_out, int32_t *n_colours_out);

/* Release a problem's device memory.  E_BUSY while a job still uses it. */
int pbit_unload_problem(pbit_ctx *ctx, uint64_t problem);

/* Number of spins N of a loaded problem, or a negative error code. */
int64_t pbit_problem_spins(pbit_ctx *ctx, uint64_t problem);

/* ---- annealing (Sec. 1.3.1 classical annealing; Sec. 1.3.3 replicas) ---- */

typedef struct {
    const double *beta;       /* [n_sweeps]: beta[s] is used for sweep sweep_offset + s; finite, >= 0 */
    int32_t n_sweeps;         /* >= 0 */
    int32_t sweep_offset;     /* >= 0: absolute index of the first sweep (resume) */
    int32_t n_replicas;       /* 1 .. 2^30 */
    int32_t replica_offset;   /* >= 0, multiple of 4: global index of replica 0 (slicing) */
    uint64_t seed;
    const int8_t *init_spins; /* host [R][N] +-1, or NULL for the Philox random start */
    int32_t trace_every;      /* 0: no trace; k > 0: record every replica's energy after
                                 sweeps k, 2k, ... (n_sweeps / k snapshots) */
    int32_t has_target;       /* nonzero: stop after the first checked sweep with min_r E_r <= target */
    int64_t target_energy;
} pbit_anneal_desc;

typedef struct {
    int8_t *spins;            /* caller [R][N] or NULL: final spins */
    int64_t *energies;        /* caller [R] or NULL: final energies */
    int64_t best_energy;      /* out: min_r E_r */
    int32_t best_replica;     /* out: lowest local replica index reaching best_energy */
    int32_t sweeps_done;      /* out: sweeps run (n_sweeps unless the target stopped it) */
    int64_t *energy_trace;    /* caller [trace_cap][R] or NULL */
    int32_t trace_cap;        /* rows available in energy_trace */
    int32_t trace_len;        /* out: rows written */
    int8_t *spin_trace;       /* caller [trace_cap][R][N] or NULL: spins at each traced sweep */
} pbit_result;

/* Run the anneal and wait for it.  When has_target is set the target is
 * tested after every traced sweep (every sweep if trace_every is 0) and the
 * run stops after the first sweep that meets it.
 * Errors: E_ARG, E_RANGE (beta), E_HANDLE, E_NOMEM, E_DEVICE. */
int pbit_anneal(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, pbit_result *result);

/* Device-memory variant: spins and energies live in device memory the caller
 * owns (e.g. torch tensors) and the work runs on `hip_stream` (a hipStream_t,
 * NULL for the context's own stream).  d_spins is int8 [R][N]: read as the
 * initial spins when `spins_in` is nonzero (desc->init_spins must then be
 * NULL), and always overwritten with the final spins.  d_energies is int64
 * [R] or NULL.  Returns after the work on the stream has finished.  Traces and
 * targets are not available here (E_ARG if requested). */
int pbit_anneal_dev(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc,
                    void *d_spins, int32_t spins_in, void *d_energies, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): pbit_anneal_dev with
 * the same arguments, results and errors, whose working buffers (the kernels'
 * spin layout, energy accumulators, threshold table) are carved from a static
 * device array of PBIT_NOALLOC_SCRATCH_BYTES instead of the context's
 * allocations.  The call itself allocates nothing on the device and creates no
 * events; the biclique kernel is the one already timed for the shape on this
 * context, else the bit or DMA tile without timing, and a cube that both
 * one-launch-per-half-sweep kernels can take runs the matrix-core half-sweep for
 * at most 1024 replicas, else the streaming stencil.  Requests whose buffers
 * exceed the array return E_UNSUPPORTED before any work is enqueued (the bytes
 * needed are about N x R for the cube and graphs, (na + nb) x R x 9/8 for the
 * biclique, plus 4 S x (max |I| + 1) for the table).  The array lives on every
 * device the library runs on until the process ends; calls on one device share
 * it and the library runs them one at a time (each returns after its work on
 * the stream has finished), so nothing of an earlier call's contents leaks into
 * a later one: buffers that must start at zero are cleared by each call. */
#define PBIT_NOALLOC_SCRATCH_BYTES (64u << 20)
int pbit_anneal_dev_noalloc(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, void *d_spins,
                            int32_t spins_in, void *d_energies, void *hip_stream);

/* Energies of R host configurations [R][N] into out[R] (computed on the GPU). */
int pbit_energy(pbit_ctx *ctx, uint64_t problem, const int8_t *spins, int32_t R, int64_t *out);

/* ---- batched anneals (Sec. 1.3.3: many independent runs) ------------------ */

/* Many independent jobs share persistent kernels: each job is cut into replica
 * tiles (4, 8 or 16 replicas of a whole cube or general graph, or 32 or 64
 * replicas of both sides of a biclique, 128 with spins held as bits) that never
 * need each other, and every workgroup keeps taking (job, tile, sweep range)
 * items from a device queue with its tile's spins held in LDS.  Results are
 * identical to pbit_anneal for the same job, whatever it is batched with.
 * Batched jobs need a cube or a general graph of at most 38,912 spins (a
 * 4-replica tile in LDS) or a biclique with na_p + nb_p <= 4,096 padded sites
 * (E_UNSUPPORTED otherwise).  When a job
 * has a target or a trace, its energies are checked every trace_every sweeps,
 * or every PBIT_CHECK_SWEEPS sweeps when trace_every is 0, and a target stops
 * the job after the first checked sweep that meets it. */
#define PBIT_CHECK_SWEEPS 100

typedef struct {
    uint64_t problem;
    const pbit_anneal_desc *desc;
    pbit_result *result;      /* filled as by pbit_anneal (spin_trace is not supported) */
} pbit_batch_job;

/* Tile sizes of batched jobs.  Where a job's shape can take more than one tile
 * size, the library times one tile of each (a couple of the job's sweeps on
 * scratch memory) when the shape is first seen and no round is in flight, and
 * keeps the size whose tiles cost the least device time per job; the choice is
 * cached per (problem kind, sides or spins, threshold width, replicas rounded up
 * to a power of two, operand mode).  PBIT_TILE_TUNE=0 at context creation keeps
 * the fixed rule (the widest tile the replicas fill).  Results do not depend on
 * the tile size.  Writes the number of timings run and of cached shapes. */
int pbit_profile_tiles(pbit_ctx *ctx, int64_t *tunings, int32_t *shapes);

/* Run all jobs and wait for them.  A job whose device memory does not fit the
 * budget while no other job runs fails the call with E_NOMEM; the call's other
 * jobs are then withdrawn (their results may be partly written). */
int pbit_anneal_batch(pbit_ctx *ctx, const pbit_batch_job *jobs, int32_t n_jobs);

/* ---- serving: continuous batching of anneal jobs ------------------------- */

/* Queue an anneal job.  The descriptor, beta and init spins are copied.  A job
 * is admitted to the GPU when its device memory fits the context's budget and
 * fewer than max_jobs jobs are running; jobs that arrive while others run join
 * the next round of the persistent kernels, so their work overlaps on the
 * device.  The device state of an admitted job (couplings, spins, RNG
 * counters, thresholds) stays resident until it completes.  Writes a job id.
 * Errors: E_ARG, E_RANGE, E_HANDLE, E_BUSY (queue full), E_NOMEM (the job can
 * never fit the budget), E_UNSUPPORTED (shape not batchable). */
int pbit_submit(pbit_ctx *ctx, uint64_t problem, const pbit_anneal_desc *desc, uint64_t *job_out);

/* PBIT_PENDING while the job is queued or running; PBIT_OK once it is done,
 * after filling `result` (same fields as pbit_anneal; spin_trace not
 * supported); the job id is then retired.  E_HANDLE for unknown ids.  E_NOMEM
 * (the id is retired, `result` untouched) when the job reached the head of the
 * queue but its device memory did not fit the budget while no job was running:
 * memory held by problems, by other calls' scratch or by finished jobs not yet
 * polled is never freed by the scheduler, so the job cannot wait for it. */
int pbit_poll(pbit_ctx *ctx, uint64_t job, pbit_result *result);

/* Drive the scheduler without waiting: harvest a finished round, admit queued
 * jobs, launch the next round.  Also done inside pbit_poll. */
int pbit_progress(pbit_ctx *ctx);

/* Scheduler limits of a context: queue capacity, concurrently running jobs and
 * sweeps per round (0 keeps the current value). */
int pbit_serve_config(pbit_ctx *ctx, int32_t max_queue, int32_t max_running, int32_t round_sweeps);

/* ---- profiling -------------------------------------------------------------- */

/* Time the sweep kernels without an external profiler (0 = off): a window of
 * min(8, every) consecutive half-sweep launches, starting at every `every`-th
 * launch of an anneal, is bracketed by one pair of HIP events recorded on the
 * stream the launches run on; pbit_profile_read returns the summed device time
 * of the windows and the number of launches inside them. */
int pbit_profile_enable(pbit_ctx *ctx, int32_t every);

/* Device time and number of the bracketed half-sweep launches of problem kind
 * `kind` (PBIT_EA3D, PBIT_BICLIQUE or PBIT_GRAPH) since the last reset; `reset` nonzero
 * clears the counters after reading. */
int pbit_profile_read(pbit_ctx *ctx, int32_t kind, double *total_ms, int64_t *launches, int32_t reset);

/* The biclique half-sweep kernel the latest biclique anneal on this context ran
 * (0 before any): 1 = 64 x 64 tiles from global memory (any side), 2 = 128 x 128
 * tiles staged in LDS by the global-to-LDS DMA (sides padded to 128), 3 = spins
 * held as bits, tiles of 64 sites x 256, 128 or 64 replicas (sides padded to 128,
 * replicas to 256), 4 = sides of at most 512 held in LDS with their couplings for
 * runs of sweeps per launch, in slices of 16 or 8 replicas.  The library times the
 * kernels the shape can take (kernel 3 in each replica tile that divides the padded
 * replica count, kernel 4 in both slice widths) on the first anneal of a shape and
 * keeps the fastest, unless PBIT_BQ_VARIANT (1..4) names a kernel, PBIT_BQ_BITS_RT
 * (64, 128, 256) a replica tile or PBIT_BQ_SLAB_RS (16, 8) a slice width, when the
 * context is created; a named kernel the shape cannot take falls back to the
 * timed choice.  All give the same spins.  *variant is written on success only. */
int pbit_profile_variant(pbit_ctx *ctx, int32_t *variant);

/* Graph use of pbit_anneal_dev on this context.  With PBIT_GRAPH=1 set when the
 * context is created, the sweep launches of pbit_anneal_dev are captured into
 * one HIP graph, instantiated and launched; the executable graph is kept and
 * replayed by later calls that launch the same kernels with the same arguments
 * (same problem, schedule, sweep and replica ranges, seed, kernel path and
 * working buffers).  Results are the same as without the graph.  Writes the
 * number of captures and of graph launches so far (either pointer may be NULL). */
int pbit_profile_graph(pbit_ctx *ctx, int64_t *captures, int64_t *launches);

/* The cube path of the latest cube anneal on this context (0 before any): 1 = the
 * streaming stencil, one launch per half-sweep; 2 = the LDS-resident form, the
 * whole lattice of 16 replicas per workgroup for runs of sweeps, taken for
 * cubes of at most 8192 sites; 3 = the fields of 32 sites x 32 replicas as int8
 * MFMAs over blocks of neighbour sites, one launch per half-sweep, possible for
 * cubes whose colour classes split into tiles of 32 sites with at most 8
 * neighbour blocks each (every cube with Lx = 32, for one).  By default a cube of
 * more than 8192 and at most 2^21 sites that allows path 3 takes whichever of
 * paths 1 and 3 ran faster when the first anneal of that shape and replica count
 * (rounded up to 128) on this context timed four half-sweeps of each; without
 * allocation (pbit_anneal_dev_noalloc) there is no timing and path 3 is taken
 * for at most 1024 replicas.  When the context is created, PBIT_EA_STREAM=1
 * selects path 1 for every cube, PBIT_EA_MFMA=1 path 3 wherever it can run,
 * PBIT_EA_MFMA=0 never path 3 and a negative value keeps the default.  All give
 * the same spins.
 * *path is written on success only. */
int pbit_profile_ea_path(pbit_ctx *ctx, int32_t *path);

/* The general-graph path of the latest graph anneal on this context (0 before
 * any): 1 = one launch per colour class (every site of the class, 16 replicas per
 * thread); 2 = the whole graph for a tile of 16, 8 or 4 replicas held in one
 * workgroup's LDS for runs of up to 1000 sweeps per launch, taken when the graph's
 * spins for 4 replicas fit (at most 39 936 spins), with the narrowest tile that
 * fits and leaves at most two workgroups per compute unit (else the widest that
 * fits).  When the context is created, PBIT_GRAPH_SLAB=0 keeps path 1 and
 * PBIT_GRAPH_SLAB=4, 8 or 16 forces that tile width where it fits.  Both paths give
 * the same spins.  *path is written on success only. */
int pbit_profile_graph_path(pbit_ctx *ctx, int32_t *path);

/* The ceilings the sweep kernels are measured against, each timed as a kernel of
 * its own over `reps` launches (after one warm-up launch) on the context's
 * stream.  *ms_per_launch receives the mean launch time and *work_per_launch
 * the work one launch does:
 *   PBIT_PROBE_PHILOX  `size` Philox4x32-10 blocks per thread (the counter layout of
 *                      the sweep), 8 workgroups of 256 threads per CU; work = words drawn;
 *   PBIT_PROBE_COPY    a device copy of `size` bytes between two buffers, one 16-byte
 *                      element per thread, each launch reading what the one before wrote;
 *                      work = bytes read plus bytes written (at most 64 GiB);
 *   PBIT_PROBE_MFMA    `size` steps of four independent v_mfma_i32_32x32x32_i8 chains
 *                      per wave, operands in registers, 8 waves per CU; work = int8
 *                      operations (two per multiply-add).
 * Uses the context's scratch memory.  Errors: E_ARG, E_NOMEM, E_DEVICE. */
enum { PBIT_PROBE_PHILOX = 1, PBIT_PROBE_COPY = 2, PBIT_PROBE_MFMA = 3 };
int pbit_probe(pbit_ctx *ctx, int32_t probe, int64_t size, int32_t reps, double *ms_per_launch,
               double *work_per_launch);

/* ---- host-side helpers (no GPU needed) ---------------------------------- */

/* The uint32 minority-threshold table Tm[s][a], s < S, a <= A, as the library
 * builds it on the host for the device (see the decision rule above). */
int pbit_threshold_table(const double *beta, int32_t S, int32_t A, uint32_t *out);

/* The greedy colouring pbit_load_graph uses when no colouring is given
 * (host only).  Writes colour[n] and the number of colours. */
int pbit_greedy_colouring(int32_t n, int32_t n_bonds, const int32_t *bond_i, const int32_t *bond_j, uint8_t *colour,
                          int32_t *n_colours);

/* Library version string. */
const char *pbit_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PBIT_H */
