/*
 * hiccl.h — C ABI of a hierarchical collective executor for one MI355X (gfx950).
 *
 * Method: HiCCL (arXiv 2408.05962). A collective is composed from multicast,
 * reduction and fence primitives (Sec. 3, Listing 1), factorized onto a
 * stated multilevel hierarchy as point-to-point transfers within each level
 * (Sec. 4.2), striped (Sec. 4.3) and pipelined (Sec. 4.5), and executed
 * without a global barrier (Sec. 5.2).
 *
 * Virtual ranks. The P ranks of the hierarchy are disjoint buffers in the
 * memory of ONE GPU. Where the paper's API takes each process's own send
 * and receive pointer, this API takes an array of P per-rank buffers with
 * any offset already applied; only the entries a primitive uses are read.
 * A "transfer" is a copy in device memory; a reduction node is a fused
 * multi-operand elementwise kernel.
 *
 * Conventions for every entry point:
 *   - returns HICCL_SUCCESS (0) or a negative hiccl_result; no exception
 *     crosses the ABI; hiccl_last_error() gives a thread-local message;
 *   - a failed call leaves the communicator as it was;
 *   - a communicator is not thread-safe; calls on one communicator must be
 *     serialized by the caller.
 *
 * Ownership: user buffers stay owned by the caller and must stay valid and
 * unmoved while a communicator that names them exists. The library copies
 * rank arrays and leaf vectors at registration, and owns its schedule, its
 * device task table and (unless the caller supplies one) its workspace.
 */
#ifndef HICCL_H
#define HICCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hiccl_comm_s* hiccl_comm_t;
typedef struct hiccl_batch_s* hiccl_batch_t;
typedef struct hiccl_server_s* hiccl_server_t;

/* One virtual rank's buffer. `data` points at element 0 (device memory for
 * hiccl_run, host memory for hiccl_validate_host). `scales` is used by the
 * fp8 payload only: one float per block of 256 consecutive elements, the
 * scale of the block that starts at `data`; NULL for other types. */
typedef struct {
  void* data;
  float* scales;
} hiccl_buf_t;

typedef enum {
  HICCL_INT32 = 0,
  HICCL_FLOAT32 = 1,
  HICCL_BFLOAT16 = 2,   /* payload bf16, sums accumulated in float32 */
  HICCL_FP8_E4M3 = 3    /* OCP e4m3 payload + float32 scale per 256 elements */
} hiccl_dtype;

/* Reduction operators (Sec. 3.1 names sum, max, logical-or and others;
 * sum, max and min are provided; bf16 and fp8 support sum only). */
typedef enum { HICCL_SUM = 0, HICCL_MAX = 1, HICCL_MIN = 2 } hiccl_op;

typedef enum {
  HICCL_SUCCESS = 0,
  HICCL_ERR_INVALID_ARG = -1,
  HICCL_ERR_STATE = -2,        /* call not allowed in the communicator's state */
  HICCL_ERR_RACE = -3,         /* two primitives of one step overlap (write-write or read-write) */
  HICCL_ERR_OOM = -4,
  HICCL_ERR_HIP = -5,          /* HIP runtime error; message in hiccl_last_error() */
  HICCL_ERR_TIMEOUT = -6,      /* the executor's bounded dependency wait expired */
  HICCL_ERR_UNSUPPORTED = -7,
  HICCL_ERR_BUSY = -8          /* serving: request deferred, HBM budget or slots exhausted */
} hiccl_result;

/* Executor forms. */
typedef enum {
  HICCL_EXEC_PERSISTENT = 0,   /* one launch; tiles claimed in dependency order, progress in device counters */
  HICCL_EXEC_STAGED = 1        /* one launch per dependency stage (kernel boundaries act as fences) */
} hiccl_exec_mode;

/* Claim order of the task table. */
typedef enum {
  HICCL_ORDER_STAGE = 0,       /* by dependency stage, then program order */
  HICCL_ORDER_PROGRAM = 1,     /* program order (primitive, branch, channel) */
  HICCL_ORDER_CHANNEL = 2,     /* pipeline channel first, then stage: each channel's intermediates are
                                  consumed soon after they are produced (cache locality) */
  HICCL_ORDER_CRITICAL = 3     /* by dependency stage, then longest chain of successors first: the
                                  schedule of the step counts of Sec. 4.6 when every rank has one
                                  link; on one GPU it separates hops that read one source, so the
                                  stage order (which keeps them together) is the default */
} hiccl_order;

/* ---------------------------------------------------------------- lifecycle */

/* Create a communicator over `nranks` virtual ranks carrying `dtype`
 * elements: the Comm<T> object of Listings 1 and 2, whose element type is
 * the template argument there (Sec. 3.2 builds every collective on one
 * such object). Defaults: hierarchy {nranks} (direct, Sec. 6.3's
 * non-hierarchical baseline), stripe 1, ring 1, pipeline 1, as the
 * optimization parameters of Sec. 4.1 before they are set. Errors:
 * INVALID_ARG for nranks < 1 or an unknown dtype; OOM. */
int hiccl_comm_create(int nranks, int dtype, hiccl_comm_t* out);

/* Free the communicator, its schedule, its device tables and its own
 * workspace. Blocks until a run in flight has finished. NULL is accepted. */
int hiccl_comm_destroy(hiccl_comm_t comm);

/* --------------------------------------------------------------- composition */

/* Register the multicast M(root, leaves, count) of Sec. 3.1: rank `root`'s
 * `count` elements at send[root] are replicated to recv[j] for every j in
 * leaves[0..nleaves). `send` and `recv` are arrays of nranks entries.
 * A leaf equal to the root receives a local copy unless send[root] and
 * recv[root] are the same address (in place).
 * Errors: INVALID_ARG (rank out of range, duplicate leaf, NULL buffer,
 * fp8 count not a multiple of 256, partially overlapping in-place buffers),
 * STATE (after hiccl_init), RACE (overlaps a primitive of the current step). */
int hiccl_add_multicast(hiccl_comm_t comm, const hiccl_buf_t* send, const hiccl_buf_t* recv,
                        size_t count, int root, const int* leaves, int nleaves);

/* Register the reduction R(leaves, root, count, op) of Sec. 3.1: the
 * elementwise `op` of send[i][0..count) over i in leaves is written to
 * recv[root]. One leaf makes a point-to-point copy (the unary operation
 * omitted). Operands are combined in a fixed, schedule-determined order,
 * so results are reproducible bit for bit. Errors as hiccl_add_multicast,
 * plus UNSUPPORTED for max/min on bf16 or fp8. */
int hiccl_add_reduction(hiccl_comm_t comm, const hiccl_buf_t* send, const hiccl_buf_t* recv,
                        size_t count, const int* leaves, int nleaves, int root, int op);

/* Close the current step (Sec. 3.3). Primitives after the fence depend on
 * those before it only where their memory ranges overlap; there is no
 * barrier. Errors: STATE after init. */
int hiccl_add_fence(hiccl_comm_t comm);

/* ------------------------------------------------------ optimization space */

/* Hierarchy factors, highest level first (Sec. 4.1 item 1, Sec. 4.2);
 * their product must equal nranks. Consecutive ranks fill the innermost
 * groups. Setting a parameter after init discards the plan (init again). */
int hiccl_set_hierarchy(hiccl_comm_t comm, const int* factors, int nlevels);

/* Striping factor s (Sec. 4.1 item 3, Sec. 4.3). Must divide some group
 * size of the hierarchy, else init fails with INVALID_ARG. Default 1. */
int hiccl_set_stripe(hiccl_comm_t comm, int s);

/* Ring length n across top-level groups (Sec. 4.4). n = 1 is the tree.
 * n > 1 must make nranks / n the size of a group of the hierarchy (n is a
 * product of leading factors), and the stripe factor must divide that
 * group; hiccl_init returns INVALID_ARG otherwise. Default 1. */
int hiccl_set_ring(hiccl_comm_t comm, int n);

/* Pipeline depth m (Sec. 4.1 item 5, Sec. 4.5): every branch is split into
 * m channels. Default 1. */
int hiccl_set_pipeline(hiccl_comm_t comm, int m);

/* One rank's share (not a paper parameter: a measurement aid). With
 * rank >= 0, hiccl_init plans only the tasks whose output lies in that
 * virtual rank's memory (its receive buffers or its workspace region): the
 * work one GPU would do if every rank were its own GPU and each GPU ran the
 * hops and reduce nodes it receives, pulling remote operands (the IPC get
 * of Sec. 5.1). Edges from
 * tasks of other ranks are dropped and the remaining stages renumbered, so
 * the kept tasks read whatever their inputs hold when they run; the result
 * is the collective's only where those inputs already hold their final
 * values (for example after a run of the full plan on the same workspace).
 * Byte accounting covers the kept tasks. hiccl_validate_host returns
 * HICCL_ERR_STATE for such a plan. rank = -1 (default) plans the whole
 * collective; values outside [-1, nranks) return INVALID_ARG. Like the
 * other set calls it discards an existing plan. */
int hiccl_set_share(hiccl_comm_t comm, int rank);

/* Executor launch options (not a paper parameter): form (hiccl_exec_mode),
 * tile size in bytes (work unit of one workgroup; 0 = default: 64 KiB for
 * the persistent executor, 112 KiB for its fp8 tables, 32 KiB for stage
 * launches; at most 1 GiB;
 * rounded to whole 16-byte vectors and whole fp8 scale blocks; hiccl_init
 * returns INVALID_ARG if a plan would need 2^31 tiles or more), grid (workgroups of the
 * persistent launch, or of each stage launch; 0 = default: one per compute
 * unit persistent; staged, one per compute unit for an int32 / float32 stage
 * whose tiles share no source, two per compute unit otherwise), claim order
 * (hiccl_order). */
int hiccl_set_exec(hiccl_comm_t comm, int mode, size_t tile_bytes, int grid, int order);

/* ------------------------------------------------------------------ init */

/* Factorize every primitive (striping, ring, tree — in that order, Sec. 4.4
 * last paragraph), split into channels, derive the dependency DAG from
 * memory-range overlaps across fences, order and tile the tasks, and size
 * the workspace. Host-only; the device tables are uploaded on the first
 * run (memoized, Sec. 5.2). Errors: INVALID_ARG (bad parameters),
 * STATE (already initialized). */
int hiccl_init(hiccl_comm_t comm);

/* Bytes of device workspace the plan needs: the intermediate buffers of
 * the factorized schedule, i.e. the partial sums of reduction nodes held
 * by staging ranks (Sec. 4.2) and the stripes a striped multicast stages
 * on its owners (Sec. 4.3). The paper allocates these inside its
 * persistent communicator at initialization (Sec. 5.2); here the caller
 * may supply them. Errors: STATE before hiccl_init; INVALID_ARG for NULL. */
int hiccl_workspace_size(hiccl_comm_t comm, size_t* bytes);

/* Use caller-owned device memory (>= hiccl_workspace_size bytes, 256-byte
 * aligned) as that workspace instead of a library allocation (Sec. 5.2's
 * buffers, owned by the caller). The memory must stay valid while the
 * communicator exists and must not be used by anything else while a run is
 * in flight. Frees uploaded device tables (they are rebuilt on the next
 * run). Errors: STATE before hiccl_init; INVALID_ARG if too small or
 * misaligned. */
int hiccl_set_workspace(hiccl_comm_t comm, void* dptr, size_t bytes);

/* --------------------------------------------------------------- execution */

/* start() of Listing 2: enqueue the whole collective on `stream` (a
 * hipStream_t; NULL = default stream) and return. The first call uploads
 * the task table. Re-running on the same stream is ordered; a run on a
 * second stream while one is in flight returns STATE. Errors: STATE (not
 * initialized), HIP, OOM. */
int hiccl_run(hiccl_comm_t comm, void* stream);

/* wait() of Listing 2: block the host until the last run's buffers may be
 * reused. Returns TIMEOUT if the executor gave up a dependency wait. After
 * hiccl_run_static it synchronizes that run's stream and reads the status
 * word in the device's static scratch (the last static run's on the device).
 * Debug check: while the environment variable HICCL_DEBUG is non-zero, this
 * call (and hiccl_batch_wait) also reads back every counter of the task
 * table and returns STATE if one is not where the next run expects it
 * (dependency, tile and claim counters zero, task counts restored). */
int hiccl_wait(hiccl_comm_t comm);

/* Size of the static device scratch of hiccl_run_static: 64 MiB, held by
 * every GPU the library runs on from its first such call until the
 * process ends. */
#define HICCL_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hiccl_run
 * without any allocation. The communicator's task table, dependency
 * counters and workspace live in a static device array of
 * HICCL_STATIC_SCRATCH_BYTES per GPU instead of library allocations; the
 * caller still passes the input and output buffers (at registration).
 * A call copies the table (built on the host at the first call and kept
 * with the communicator) into the array on `stream`, which also resets
 * every counter, unless the array still holds this communicator's table
 * from its previous static call on the device; then it launches the same
 * kernels as hiccl_run. It calls no hipMalloc / hipFree and ignores a
 * workspace set by hiccl_set_workspace.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents: calls that overlap on one GPU (two streams, or the
 * device request ring of a server) race and give undefined results, so the
 * caller orders them. hiccl_wait follows the latest static run. Errors:
 * STATE (not initialized, or a run of this communicator in flight on
 * another stream), INVALID_ARG (the plan's workspace and tables need more
 * than HICCL_STATIC_SCRATCH_BYTES; checked before any device call), HIP. */
int hiccl_run_static(hiccl_comm_t comm, void* stream);

/* Workgroups of the next runs (0 = the default of hiccl_set_exec), without re-planning.
 * A smaller grid lets several collectives share the device at once. */
int hiccl_set_grid(hiccl_comm_t comm, int grid);

/* Tile claiming of the persistent executor (not a paper parameter): the
 * task table is dealt round-robin into `queues` queues (1..8; 0 = 8), each
 * claimed `batch` tiles per atomic (0 = 4). A single queue keeps progress
 * independent of how many workgroups are resident at once (use it when
 * other kernels share the device); several queues cut counter contention. */
int hiccl_set_claim(hiccl_comm_t comm, int queues, int batch);

/* Bounded-wait budget of the persistent executor, in polls of a dependency
 * counter (default 2^22, a few seconds). Expiry aborts the run cleanly:
 * every workgroup exits and hiccl_wait returns TIMEOUT. */
int hiccl_set_spin_limit(hiccl_comm_t comm, uint32_t polls);

/* Task timeline of the persistent executor (the pipelining picture of
 * Sec. 4.5: which transfers of which channel overlap in time). With trace on
 * (1), runs of this communicator on the persistent executor stamp, for every
 * task, the device clock when its first tile starts and when its last tile
 * retires; off (0, the default) they stamp nothing. Changing it drops the
 * uploaded tables (the next run uploads them again). INVALID_ARG for other
 * values. */
int hiccl_set_trace(hiccl_comm_t comm, int on);
/* The last traced run's timeline, after hiccl_wait: start_ns[i] / end_ns[i]
 * for plan task i (the order of hiccl_plan_tasks), in ns from the earliest
 * task start of that run. Arrays of ntasks entries, ntasks = the plan's task
 * count (INVALID_ARG otherwise). STATE if trace is off, the executor is not
 * the persistent one, or the communicator has no traced run of its own (a
 * batch or hiccl_run_static run is not traced). After a run that gave up a
 * dependency wait (TIMEOUT) the tasks it did not reach keep the stamps of an
 * earlier run. */
int hiccl_trace_tasks(hiccl_comm_t comm, uint64_t* start_ns, uint64_t* end_ns, size_t ntasks);

/* ------------------------------------------------------------- accounting */

/* Communication volume of the plan, per hierarchy level: the per-level
 * form of the communication matrix of Sec. 4.5 (bytes between every pair
 * of ranks, summed by the level at which the pair first differs). Its
 * top-level entry is the inter-node volume behind the throughput bounds of
 * Table 3, which the tree factorization keeps at the minimum the collective
 * needs (Sec. 4.2). Logical bytes per
 * level of ANY accounting hierarchy `acct` (product = nranks; NULL / 0 =
 * the communicator's own), for the initialized plan: level_bytes[0] = local copies,
 * level_bytes[k] = transfers whose endpoints first differ at depth k
 * (1 = highest). A reduction node counts one transfer per operand held by
 * another rank. hbm_read / hbm_written = bytes the executor reads and
 * writes in device memory (every task; fp8 scales included). Any output
 * pointer may be NULL. */
int hiccl_query_bytes(hiccl_comm_t comm, const int* acct, int nacct, uint64_t* level_bytes,
                      uint64_t* hbm_read, uint64_t* hbm_written);

#define HICCL_INFO_MAX_SRC 16

/* One task of the plan, as exported for inspection. */
typedef struct {
  int kind;            /* 0 copy, 1 reduce */
  int prim;            /* registration index of the primitive */
  int step;            /* fence-delimited step of that primitive */
  int stripe;          /* stripe index (0 if not striped) */
  int channel;         /* pipeline channel */
  int stage;           /* dependency depth: 0 for tasks with no predecessor */
  int dst_rank;        /* rank that owns the written buffer */
  int dst_workspace;   /* 1 if the destination is library workspace */
  int nsrc;
  int src_rank[HICCL_INFO_MAX_SRC];
  int npred;           /* predecessors in the DAG */
  int ring_step;       /* 0 for tree hops; ring position otherwise */
  uint64_t count;      /* elements */
  uint64_t offset;     /* element offset inside the primitive */
} hiccl_task_info_t;

typedef struct {
  uint64_t ntasks, ntiles, nedges, nstages;
  uint64_t workspace_bytes;
  uint64_t hbm_read, hbm_written;
  uint64_t tile_elems;
} hiccl_plan_info_t;

int hiccl_plan_info(hiccl_comm_t comm, hiccl_plan_info_t* info);

/* Copy up to `cap` task descriptions, in claim order, into `out`. */
int hiccl_plan_tasks(hiccl_comm_t comm, hiccl_task_info_t* out, size_t cap, size_t* n);
/* The dependency edges of the plan (Sec. 3.3 fences, Sec. 4.5 channels):
 * edge e says task to[e] may start only after task from[e] has finished
 * (indices in the order of hiccl_plan_tasks). Copies up to `cap` edges;
 * *n = the total. INVALID_ARG for NULL outputs with cap > 0, STATE before
 * hiccl_init. */
int hiccl_plan_edges(hiccl_comm_t comm, uint32_t* from, uint32_t* to, size_t cap, size_t* n);

/* Schedule checker (debugging aid; never used by hiccl_run): executes the
 * plan on HOST memory — the registered buffers must be host pointers — in
 * `norders` random dependency-respecting orders with poisoned workspace,
 * so a missing dependency edge shows up as a wrong result. Results of the
 * last order are left in the receive buffers. */
int hiccl_validate_host(hiccl_comm_t comm, uint64_t seed, int norders);

/* ---------------------------------------------------------------- batching */

typedef enum {
  HICCL_BATCH_PERSISTENT = 0,  /* all task tables merged into one persistent launch, members in groups
                                  of about 1 GiB of executed bytes, claimed group after group */
  HICCL_BATCH_GRAPH = 1,       /* captured once into a hipGraph and replayed: 4 parallel branches,
                                  balanced by executed bytes, each running its collectives as stage
                                  launches on a quarter of the device */
  HICCL_BATCH_SERIAL = 2,      /* one launch per collective on the stream (reference form) */
  HICCL_BATCH_PERSISTENT_SJF = 3, /* one merged launch, smallest collectives claimed first (grouped
                                     the same way, in order of executed bytes) */
  HICCL_BATCH_STAGED = 4          /* task tables merged by dependency stage; one launch per stage for
                                     a group of members (about 4 GiB of executed bytes), group after group
                                     (completion = end of a collective's last stage launch) */
} hiccl_batch_mode;
/* The merged forms (PERSISTENT, PERSISTENT_SJF, STAGED) run their members in
 * groups so that a collective's stages run close together and read what the
 * previous stage wrote from the caches. The environment variable
 * HICCL_BATCH_GROUP_MB, read when a batch is built, overrides the group size
 * (MiB of executed bytes; 0 = all members in one group). */

/* Group initialized communicators (any mix of dtypes and hierarchies) into
 * one batch. Members run with no ordering between them, so they must be
 * disjoint: no communicator twice, and no member may write caller memory
 * (or a caller-provided workspace) that another member reads or writes;
 * INVALID_ARG otherwise (read-read sharing is fine). The communicators must
 * outlive the batch and must not run on their own, or in another batch,
 * while a run of this one is in flight. Re-planning a member (any set call
 * that discards its plan, hiccl_set_claim, hiccl_set_workspace) makes the
 * batch stale: hiccl_batch_run then returns STATE. */
int hiccl_batch_create(const hiccl_comm_t* comms, int n, int mode, hiccl_batch_t* out);
/* Enqueue the batch on `stream` and return. STATE if a member changed since
 * creation or the batch is in flight on another stream. */
int hiccl_batch_run(hiccl_batch_t batch, void* stream);
int hiccl_batch_wait(hiccl_batch_t batch);
/* Completion times (ns, relative to the batch start) of each collective of
 * the last run. Persistent forms: the device clock at the moment its last
 * task retired. Graph / serial: the device clock when its last launch
 * finished. Staged: stream events, the end of its last stage launch. An
 * empty collective (count 0: no task) reports 0. `ns` has n entries. */
int hiccl_batch_times(hiccl_batch_t batch, uint64_t* ns, int n);
int hiccl_batch_destroy(hiccl_batch_t batch);

/* Run `n` initialized communicators as one batch of form `mode`
 * (hiccl_batch_mode) on `stream` and return at once: many collectives of
 * one training or serving step issued together. The batch is built on the
 * first call for this list of members and form (the same rules as
 * hiccl_batch_create) and memoized, as the paper memoizes a collective's
 * schedule when it is initialized (Sec. 5.2): later calls with the same
 * list reuse its uploaded table. hiccl_wait on any member then waits for
 * the whole batch (TIMEOUT if a dependency wait expired); a later hiccl_run
 * of a member alone leaves the batch. The memoized batch is dropped when a
 * member is re-planned or destroyed; at most 16 are kept (the oldest goes).
 * Errors: as hiccl_batch_create / hiccl_batch_run; STATE if a member is in
 * flight in another batch on another stream. */
int hiccl_run_batch(const hiccl_comm_t* comms, int n, void* stream, int mode);

/* Autotuner: times every (stripe, pipeline, tile) candidate on `stream`
 * (`reps` runs each after one warm-up) and re-initializes the communicator
 * with the fastest. Candidates that are invalid for the hierarchy are
 * skipped. Writes the choice and its median time (microseconds). */
int hiccl_autotune(hiccl_comm_t comm, const int* stripes, int nstripes, const int* pipes, int npipes,
                   const size_t* tiles, int ntiles, int reps, void* stream, int* best_stripe,
                   int* best_pipe, size_t* best_tile, double* best_us);

/* Model-guided autotuner (prior in the spirit of the cost model of Sec. 4.6):
 * every candidate is planned on the host to obtain its executed bytes,
 * tiles and dependency stages; t = bytes / BW + a * tiles + b * stages + c
 * (nonnegative cost weights) is fitted by least squares to `anchors` timed
 * candidates chosen far apart in that feature space, and only the `top`
 * best-predicted candidates are timed in addition. `measured`
 * returns how many candidates ran on the device. Otherwise as
 * hiccl_autotune. */
int hiccl_autotune_model(hiccl_comm_t comm, const int* stripes, int nstripes, const int* pipes, int npipes,
                         const size_t* tiles, int ntiles, int reps, int anchors, int top, void* stream,
                         int* best_stripe, int* best_pipe, size_t* best_tile, double* best_us, int* measured);

/* Batched-context autotuner (stripe, pipeline and chunk size chosen for a
 * batch of many collectives, Sec. 4.1 items 3 and 5 applied per class of
 * members): `cls[i]` in [0, nclasses) assigns member i to a class (for
 * example its collective type and size class). Coordinate descent over the
 * classes on the median time (of `reps` runs after a warm run) of the merged
 * launch of all `n` members in batch form `mode`: every class starts from
 * stripes[0], pipes[0], tiles[0] (put the defaults first); each sweep visits
 * the classes in turn and, per parameter, tries every other candidate with
 * the rest fixed, keeping a change that shortens the batch by more than 1 %;
 * it stops after `sweeps` sweeps or a sweep without change. Candidates that
 * some member of the class cannot plan are skipped. The members are left
 * initialized with the chosen values, which are written per class to
 * best_stripe / best_pipe / best_tile [nclasses]; best_ms = the batch's
 * median time under them. Members must satisfy hiccl_batch_create's rules.
 * Errors: INVALID_ARG (empty lists, class out of range, first candidate not
 * plannable), HIP. */
int hiccl_autotune_batch(const hiccl_comm_t* comms, int n, const int* cls, int nclasses, const int* stripes,
                         int nstripes, const int* pipes, int npipes, const size_t* tiles, int ntiles, int mode,
                         int reps, int sweeps, void* stream, int* best_stripe, int* best_pipe, size_t* best_tile,
                         double* best_ms);

/* ----------------------------------------------------------------- serving */

/* Admission and slot manager for a stream of collective requests
 * (continuous batching). Up to `slots` admitted requests run concurrently,
 * each on its own stream; the device memory a request keeps resident
 * (`footprint`: its buffers and workspace) is charged against `hbm_budget`
 * bytes from admission until it has finished. A request that arrives while
 * others run is admitted as soon as a slot and enough budget are free. */
int hiccl_server_create(size_t hbm_budget, int slots, hiccl_server_t* out);
/* Reserve a slot and `footprint` bytes for a new request. Returns BUSY when
 * no slot or not enough budget is free right now (call progress and retry),
 * INVALID_ARG when the footprint exceeds the whole budget. */
int hiccl_server_admit(hiccl_server_t srv, size_t footprint, uint64_t* ticket);
/* The stream (hipStream_t) of an admitted request's slot, for the caller's
 * own preparation work before the launch. */
int hiccl_server_stream(hiccl_server_t srv, uint64_t ticket, void** stream);
/* Start an admitted request: enqueue `comm` (initialized) on its slot. It
 * sets the request's grid (hiccl_set_grid): the executor's full default
 * when no other request is running, else about 3 x compute units / slots
 * workgroups, so that concurrent requests overlap on the device. With more
 * than one slot a persistent-executor request claims its tiles from one
 * queue for this launch (hiccl_set_claim's setting is left as it was), so
 * its progress never depends on how many of its workgroups are resident
 * beside other requests. If the launch fails, the ticket is released (slot
 * and budget) and the error returned. */
int hiccl_server_launch(hiccl_server_t srv, uint64_t ticket, hiccl_comm_t comm);
/* Admit and launch in one call: the request's footprint is the union of the
 * caller memory its primitives touch plus its workspace. Returns BUSY (with
 * nothing charged) when no slot or budget is free right now; otherwise as
 * hiccl_server_admit and hiccl_server_launch. */
int hiccl_server_submit(hiccl_server_t srv, hiccl_comm_t comm, uint64_t* ticket);
/* Retire finished requests (frees their slots and budget); non-blocking. */
int hiccl_server_progress(hiccl_server_t srv);
/* done = 1 once the request has finished; device_us = its time on the
 * device, launch to completion, from stream events. A finished ticket is
 * forgotten after this call; if its run gave up a dependency wait, the call
 * returns TIMEOUT (with done = 1). */
int hiccl_server_poll(hiccl_server_t srv, uint64_t ticket, int* done, double* device_us);
/* Block until every launched request has finished and retire them. */
int hiccl_server_drain(hiccl_server_t srv);
/* Bytes currently charged and requests currently running. */
int hiccl_server_usage(hiccl_server_t srv, size_t* used_bytes, int* running);
/* Serve the following launches from a device request ring instead of one
 * launch each. A resident launch of `grid` workgroups (0 = one per compute
 * unit; otherwise at least 2) on a stream of its own serves the ring:
 * workgroup 0 polls the ring's tail in host-coherent memory and publishes
 * new requests to the others, which execute the requests in arrival order
 * with the persistent executor's claim / wait / retire steps, one request's
 * last tiles overlapping the next one's first. hiccl_server_launch then
 * appends the communicator's uploaded table to the ring (it must use the
 * persistent executor; UNSUPPORTED otherwise), and progress / poll read
 * each request's completion word; device_us is 0 for these requests. The
 * resident launch exits after `idle_ms` (1..60000) without a new request,
 * and a later launch starts it again; while it runs, a device-wide
 * synchronization (hipDeviceSynchronize) waits for it to go idle. A
 * communicator must not run elsewhere while it is in the ring. The ring
 * holds 4096 entries; HICCL_ERR_STATE if requests are in flight or the ring
 * is already started. hiccl_server_destroy stops the ring after it has
 * served what was appended (bounded wait: TIMEOUT, with nothing freed, if
 * the resident launch does not stop within 30 s). */
int hiccl_server_start_ring(hiccl_server_t srv, int grid, int idle_ms);
int hiccl_server_destroy(hiccl_server_t srv);

/* --------------------------------------------------------- payload formats */

/* Convert `n` float32 values to the payload format on the device, in
 * stream order: bf16 (round to nearest even) into `out` (uint16 bits), or
 * e4m3 codes into `out` with one power-of-two float32 scale per 256
 * elements into `scales` (n must be a multiple of 256). */
int hiccl_to_payload(int dtype, const float* in, void* out, float* scales, size_t n, void* stream);
/* Widen a payload back to float32 on the device. */
int hiccl_from_payload(int dtype, const void* in, const float* scales, float* out, size_t n, void* stream);

/* ------------------------------------------------------------------- misc */

const char* hiccl_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int hiccl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HICCL_H */
