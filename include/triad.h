/*
 * triad.h - C ABI of the MI355X directed triad census (libtriad.so).
 *
 * The census: for a simple digraph on vertices 0..n-1, the number of vertex
 * triples in each of the 16 isomorphism classes, in the standard order
 *     [0]=003 [1]=012 [2]=102 [3]=021D [4]=021U [5]=021C [6]=111D [7]=111U
 *     [8]=030T [9]=030C [10]=201 [11]=120D [12]=120U [13]=120C [14]=210 [15]=300
 * (Sec. 3 of Chin, Marquez, Choudhury, Feo, "Scalable Triadic Analysis of
 * Large-Scale Graphs": 64 triad states condensed to 16 classes). 111D is
 * A<->B<-C (the asymmetric arc points into the mutual dyad), 111U is A<->B->C.
 *
 * Method: the Batagelj-Mrvar edge sweep (Fig. 5 of the paper): for every
 * symmetric edge {u,v} with u < v, the sorted neighbour lists N(u) and N(v)
 * are merged (Sec. 6, Fig. 8); each third vertex w is classified from the
 * direction bits of u-w and v-w (in situ, Sec. 6) when the triad is owned by
 * this edge (v < w, or u < w < v with w not adjacent to u); the edge adds
 * n - |N(u) u N(v)| triads to 012 (asymmetric u-v) or 102 (mutual u-v)
 * (steps 2.1.2-2.1.3); 003 = C(n,3) minus the rest (steps 3-5). All counts
 * are exact integers; the kernels are hand-written HIP for gfx950.
 *
 * Input graph (compact CSR of Sec. 6 / Fig. 7, direction bits kept in a
 * separate packed array):
 *   csr_offsets int64[n+1]   row x owns entries [csr_offsets[x], csr_offsets[x+1]);
 *                            csr_offsets[0] = 0, non-decreasing, csr_offsets[n] = nnz
 *   csr_nbrs    int32[nnz]   neighbour ids in [0,n), strictly increasing within a
 *                            row, no self-loops; symmetric: y in N(x) iff x in N(y)
 *   dir_flags   uint8[ceil(nnz/4)]  2 bits per entry, entry j at bits 2*(j&3) of
 *                            byte j>>2: bit0 = arc row->neighbour, bit1 = arc
 *                            neighbour->row; never 0; mirrored between (x,y) and (y,x)
 * Limits: 0 <= n < 2^30, every degree < 2^31, nnz < 2^40.
 *
 * Output: out_u64[0..15] in the order above. Counts [1..15] are exact. 003 can
 * exceed 2^64 (from n = 4,801,281): out_u64[0] then holds 003 mod 2^64, the
 * status is TRIAD_OK_003_WRAPPED and the high word is returned where the entry
 * point offers it. For n < 3 every count is 0.
 *
 * Ownership: inputs are borrowed read-only for the duration of the call and
 * never retained or freed. On any error status (< 0) nothing is written to the
 * outputs and triad_last_error() describes the cause (thread-local string).
 * Calls are reentrant; calls on one stream run in stream order.
 */
#ifndef TRIAD_H
#define TRIAD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRIAD_ABI_VERSION 1

enum triad_status {
  TRIAD_OK = 0,
  TRIAD_OK_003_WRAPPED = 1, /* success; 003 >= 2^64 (see above) */
  TRIAD_EINVAL = -1,        /* null pointer, negative or too-large size, bad option */
  TRIAD_EUNSORTED = -2,     /* a row is not strictly increasing (includes duplicates) */
  TRIAD_ESELFLOOP = -3,     /* a vertex lists itself */
  TRIAD_EASYM = -4,         /* CSR not symmetric or flags not mirrored (full validation) */
  TRIAD_ERANGE = -5,        /* neighbour id outside [0,n), offsets not monotone or not
                               ending at nnz, or a flag equal to 0 */
  TRIAD_ENOMEM = -6,        /* device or host allocation failed */
  TRIAD_EDEVICE = -7        /* no usable HIP device, or a HIP runtime error */
};

/* Order of the census work queue. Whole tasks are claimed in batches of 64
 * consecutive queue positions; a schedule keeps CSR order for the bulk of the
 * queue (tasks of one row u share N(u) in cache) and orders its last batches
 * (the last 1/10 of them, at least 4,096 and at most all) costliest first,
 * binned by the batch's summed cost key, when the keys predict a batch at the
 * very end costly enough to delay the census (see triad_opts.tail_share);
 * otherwise CSR order stays. */
enum triad_schedule {
  TRIAD_SCHED_PLAIN = 0,     /* tasks in CSR order */
  TRIAD_SCHED_HEURISTIC = 1, /* last batches costliest first by the summed merge lengths
                                of their tasks (ids of N(u) above u plus ids of N(v)
                                from u on) */
  TRIAD_SCHED_LEARNED = 2    /* last batches costliest first by the learned cost model's
                                predicted cycles, summed over the batch */
};

/* Device time of each stage of one census call, in milliseconds (HIP events
 * on the call's stream). */
typedef struct triad_timing {
  float prep_ms;     /* pack ids with direction bits + validation */
  float tasks_ms;    /* task enumeration (scan) and scheduling */
  float census_ms;   /* the merge/classify kernel */
  float finalize_ms; /* reduction and the null count */
  int64_t tasks;     /* number of (u,v) tasks, u < v = symmetric edges */
  int64_t hub_tasks; /* tasks split across several wavefronts */
  int64_t items;     /* work items after splitting */
  int64_t waves;     /* wavefronts of the persistent census launch */
} triad_timing;

/* Options (a zeroed struct gives the defaults). */
typedef struct triad_opts {
  int32_t schedule;        /* enum triad_schedule */
  int32_t validate;        /* 0 = O(nnz) checks of ranges, flags, order and self-loops
                              (default), 1 = also symmetry and flag mirroring */
  int64_t hub_threshold;   /* tasks with d(u)+d(v) above this are split into chunks
                              merged by different wavefronts; 0 = default, < 0 = never */
  int64_t chunk;           /* merge entries per chunk of a split task; 0 = default */
  const float *model;      /* TRIAD_SCHED_LEARNED: device pointer to the cost-model
                              weights (TRIAD_MLP_PARAMS floats); NULL = heuristic */
  uint32_t *task_cycles;   /* optional device buffer [tasks]: receives per-task
                              wavefront cycle counts, indexed in CSR task order */
  triad_timing *timing;    /* optional host output */
  int32_t waves_per_group; /* wavefronts per workgroup (1, 2 or 4); 0 = default */
  int32_t grid_groups;     /* persistent grid size in workgroups; 0 = default */
  int32_t kernel_variant;  /* census kernel variant (LDS window and counter layout),
                              set by triad_batch_autotune; 0 = the default */
  uint64_t *wave_span;     /* optional device buffer [waves][2]: real-time clock
                              (s_memrealtime, 100 MHz) at each census wavefront's
                              start and end; size it with timing->waves of a
                              previous call or grid_groups * waves_per_group */
  int32_t tail_share;      /* schedules: the last batches are reordered only when one
                              of the last 8,192 is predicted to cost more than the
                              mean of the last 32,768 by tail_share / 10,000 of one
                              wavefront's share of the whole census; 0 = default
                              (30, i.e. 0.3%), < 0 = always */
  int32_t short_tasks;     /* batched census: 0 = tasks whose two merged lists are short
                              run several to a round (default), < 0 = every task through
                              the per-task merge rounds */
} triad_opts;

/* Census of one graph given by HOST pointers (copied to the device; the call
 * blocks until the result is on the host). Default options; the high word of
 * 003 is not returned (use triad_census_ex). */
int triad_census(int64_t n, const int64_t *csr_offsets, const int32_t *csr_nbrs, const uint8_t *dir_flags,
                 uint64_t out_u64[16]);

/* As triad_census, with options (may be NULL) and the high word of 003
 * (out_003_hi may be NULL). */
int triad_census_ex(int64_t n, const int64_t *csr_offsets, const int32_t *csr_nbrs, const uint8_t *dir_flags,
                    const triad_opts *opts, uint64_t out_u64[16], uint64_t *out_003_hi);

/* Census of one graph given by DEVICE pointers (e.g. torch tensors), enqueued
 * on `hip_stream` (a hipStream_t; NULL = the null stream). nnz must equal
 * csr_offsets[n]. Results go to d_out (device, 17 x uint64: the 16 counts,
 * then the high word of 003) and, if h_out is not NULL, to h_out (host, 17 x
 * uint64). The call waits for its own work on the stream before returning the
 * status. Scratch memory comes from the library's held blocks (see
 * triad_held_memory), allocated on first use. */
int triad_census_device(int64_t n, int64_t nnz, const int64_t *csr_offsets, const int32_t *csr_nbrs,
                        const uint8_t *dir_flags, const triad_opts *opts, void *hip_stream, uint64_t *d_out,
                        uint64_t *h_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the census of
 * triad_census_device, same arguments and results, with no allocation at all.
 * Its scratch is one static device array of TRIAD_NOALLOC_SCRATCH_BYTES per
 * GPU, held until the process ends; the call takes that GPU's copy (the
 * current device's). Options: plain schedule only, task_cycles and timing
 * NULL (else TRIAD_EINVAL). A graph whose scratch would not fit (per vertex
 * 28 B, per CSR entry about 22 B, each buffer rounded up to 256 B; for example
 * 2^20 vertices with 1.5 M entries fit) is rejected with TRIAD_EINVAL before
 * anything is launched. Every call on one GPU shares its array and leaves its
 * contents behind (each call clears what it needs): calls that overlap in
 * time on one GPU, from several threads or streams, race and their results
 * are undefined; calls in sequence are safe, since each waits for its own work
 * before returning. */
#define TRIAD_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int triad_census_device_noalloc(int64_t n, int64_t nnz, const int64_t *csr_offsets, const int32_t *csr_nbrs,
                                const uint8_t *dir_flags, const triad_opts *opts, void *hip_stream,
                                uint64_t *d_out, uint64_t *h_out);

/* The 64-state labelled census (Sec. 3: the 64 states of a triad before they
 * are condensed into 16 classes) of one graph given by DEVICE pointers, same
 * arguments as triad_census_device. The vertices of a triple are named by id
 * order, a < b < c, and its state is f_ab | f_ac << 2 | f_bc << 4 (f_xy the
 * direction flag of y in row x: bit0 = x->y, bit1 = y->x, 0 = no arc). Output
 * (d_out on the device and, if not NULL, h_out on the host): 65 x uint64, the
 * count of triples in each state 0..63, then the high word of state 0 (no
 * arc: C(n,3) minus the rest); TRIAD_OK_003_WRAPPED when that high word is not
 * zero. Condensing state s into the class of the triad code s gives the
 * census of triad_census_device. Options as there, except task_cycles,
 * kernel_variant and waves_per_group (must be 0). */
int triad_labelled_census_device(int64_t n, int64_t nnz, const int64_t *csr_offsets, const int32_t *csr_nbrs,
                                 const uint8_t *dir_flags, const triad_opts *opts, void *hip_stream,
                                 uint64_t *d_out, uint64_t *h_out);

/* Host-side validation of the input contract (no device needed). level 0 =
 * cheap checks, 1 = also symmetry and mirrored flags. Returns TRIAD_OK or the
 * error status the census would return. */
int triad_validate_host(int64_t n, const int64_t *csr_offsets, const int32_t *csr_nbrs, const uint8_t *dir_flags,
                        int32_t level);

/* ---------------------------------------------------------------- batches
 * G graphs in one concatenated CSR held in DEVICE memory: graph g owns rows
 * [vbase[g], vbase[g+1]) of csr_offsets (global entry positions) and its
 * neighbour ids are graph-local (0 .. vbase[g+1]-vbase[g]-1). Each graph must
 * satisfy the single-graph contract and have fewer than 4,801,281 vertices.
 * A plan owns the scratch memory and a captured hipGraph of the whole batched
 * census (one persistent launch); launching it replays the graph on a stream.
 * d_out receives G x 16 uint64 (graph-major). */
typedef struct triad_batch_plan triad_batch_plan;

int triad_batch_plan_create(int32_t G, int64_t nv, int64_t nnz, const int64_t *d_vbase,
                            const int64_t *d_offsets, const int32_t *d_nbrs, const uint8_t *d_flags,
                            uint64_t *d_out, const triad_opts *opts, void *hip_stream, triad_batch_plan **plan);
int triad_batch_plan_launch(triad_batch_plan *plan, void *hip_stream);
/* Waits for the last launch and reports any validation error it found. */
int triad_batch_plan_status(triad_batch_plan *plan);
void triad_batch_plan_destroy(triad_batch_plan *plan);

/* One-shot batched census (plan, launch, wait, destroy). */
int triad_census_batch(int32_t G, int64_t nv, int64_t nnz, const int64_t *d_vbase, const int64_t *d_offsets,
                       const int32_t *d_nbrs, const uint8_t *d_flags, const triad_opts *opts, void *hip_stream,
                       uint64_t *d_out);

/* Autotuner for the batched census: times the candidate launch shapes on the
 * given batch with HIP events and returns the fastest in *best (its
 * waves_per_group, grid_groups, hub_threshold and chunk fields are set).
 * If cache_path is not NULL the result is read from / appended to that JSON
 * lines file, keyed by the device name and a signature of the batch. */
int triad_batch_autotune(int32_t G, int64_t nv, int64_t nnz, const int64_t *d_vbase, const int64_t *d_offsets,
                         const int32_t *d_nbrs, const uint8_t *d_flags, void *hip_stream,
                         const char *cache_path, triad_opts *best);

/* ------------------------------------------------------ CSR construction
 * The compact CSR with direction bits (Sec. 6, Fig. 7) built on the device
 * from an arc list: d_src[i] -> d_dst[i], i < narcs (DEVICE int32 arrays,
 * endpoints in [0, n)). Self-loops are dropped and duplicate arcs merged; row x
 * lists, ascending, every y with an arc x->y or y->x, with flag bit0 = x->y
 * and bit1 = y->x (the single-graph input contract above). Outputs, DEVICE
 * memory allocated by the caller: d_offsets int64[n+1], d_nbrs int32 with room
 * for 2*narcs entries, d_flags uint8 with room for ceil(2*narcs/4) bytes (the
 * first nnz entries and ceil(nnz/4) bytes are written); *nnz_out (host)
 * receives nnz. device_ms (host, may be NULL) receives the device time of the
 * construction measured with HIP events on the stream. Limits: n < 2^30,
 * narcs < 2^31. Errors: TRIAD_EINVAL (sizes, NULL pointers), TRIAD_ERANGE (an
 * endpoint outside [0, n); no output is written), TRIAD_ENOMEM. Scratch comes
 * from the library's held blocks (see triad_held_memory), about 35 bytes per
 * arc. The call waits for its work on hip_stream before returning. */
int triad_csr_from_arcs(int64_t n, int64_t narcs, const int32_t *d_src, const int32_t *d_dst, void *hip_stream,
                        int64_t *d_offsets, int32_t *d_nbrs, uint8_t *d_flags, int64_t *nnz_out,
                        float *device_ms);

/* ---------------------------------------------------- incremental census
 * The census of a graph that changes over time, monitored at fixed intervals
 * (Sec. 3, Figs. 3-4): given the graph before a batch of arc updates (DEVICE
 * CSR as above) and its census census_in (HOST, 17 words: the 16 counts, then
 * the high word of 003), returns in census_out (HOST, 17 words, same layout)
 * the census after the batch, from the neighbour lists of the changed pairs
 * only, and, if d_offsets_new is not NULL, writes the CSR after the batch.
 * Update i (DEVICE arrays) inserts the arc d_src[i] -> d_dst[i] when
 * d_insert[i] = 1 and deletes it when 0; updates apply in order (the last
 * update of an arc decides; inserting a present arc or deleting an absent one
 * changes nothing). Outputs of the new CSR (DEVICE, caller-allocated):
 * d_offsets_new int64[n+1], d_nbrs_new int32 with room for nnz + 2*nupd
 * entries, d_flags_new uint8 with room for ceil((nnz + 2*nupd)/4) bytes;
 * *nnz_new (host) receives the new entry count. changed_pairs (host, may be
 * NULL) receives the number of vertex pairs whose arcs changed. census_in
 * must be the census of the input graph (it is not checked). Limits as for
 * triad_census_device, nnz < 2^32, nupd < 2^31. Errors: TRIAD_EINVAL,
 * TRIAD_ERANGE (an endpoint outside [0, n) or d_insert[i] > 1),
 * TRIAD_ESELFLOOP (an update of a self-loop), TRIAD_ENOMEM; nothing is written
 * on error. Returns TRIAD_OK_003_WRAPPED when the new 003 is >= 2^64. The
 * call waits for its work on hip_stream before returning; its scratch comes
 * from the library's held blocks (see triad_held_memory). */
int triad_census_update(int64_t n, int64_t nnz, const int64_t *d_offsets, const int32_t *d_nbrs,
                        const uint8_t *d_flags, int64_t nupd, const int32_t *d_src, const int32_t *d_dst,
                        const uint8_t *d_insert, const uint64_t census_in[17], uint64_t census_out[17],
                        int64_t *d_offsets_new, int32_t *d_nbrs_new, uint8_t *d_flags_new, int64_t *nnz_new,
                        int64_t *changed_pairs, void *hip_stream);

/* ------------------------------------------------- significance profile
 * Triad significance profile of a graph against a null-model ensemble (for
 * example degree-preserving randomisations of it, censused in one batch):
 * d_ensemble (DEVICE, G x 16 uint64, graph-major: the output of a batched
 * census) and real (HOST, 16 uint64: the graph's census; 003 below 2^64) give
 * per type t the z-score z_out[t] = (real[t] - mean_t) / sd_t (HOST; mean and
 * sample standard deviation of the ensemble, divisor G - 1; 0 where the
 * ensemble's counts do not vary), and sp_out (HOST) the profile: the z-scores
 * of the 13 connected types (021D ... 300) scaled to unit length, 0 for 003,
 * 012, 102 (all 0 if every connected z-score is 0). Double precision. G >= 2;
 * each type's counts must lie within 2^63 of the first graph's. Errors:
 * TRIAD_EINVAL, TRIAD_ENOMEM, TRIAD_EDEVICE. Waits for its work on hip_stream. */
int triad_significance_profile(int32_t G, const uint64_t *d_ensemble, const uint64_t real[16], double z_out[16],
                               double sp_out[16], void *hip_stream);

/* ------------------------------------------------------- learned schedule
 * Cost model: an FP32 multilayer perceptron 6 -> 32 -> 32 -> 1 with ReLU
 * hidden layers. Parameters, packed in this order: W1[32][6], b1[32],
 * W2[32][32], b2[32], W3[32], b3 (1313 floats). Input features of a task
 * (u,v), from the lengths its merge walks: with a = the ids of N(u) above u
 * and b = the ids of N(v) not below u, log2(1+x) of a, b, a+b, min(a,b),
 * max(a,b), and the number of entries of N(u) above v. Target: log2 of the
 * task's measured cycles. */
#define TRIAD_MLP_IN 6
#define TRIAD_MLP_HIDDEN 32
#define TRIAD_MLP_PARAMS (TRIAD_MLP_HIDDEN * TRIAD_MLP_IN + TRIAD_MLP_HIDDEN + \
                          TRIAD_MLP_HIDDEN * TRIAD_MLP_HIDDEN + TRIAD_MLP_HIDDEN + TRIAD_MLP_HIDDEN + 1)

/* Features of every task (CSR task order) into d_feat [tasks][6] (device). */
int triad_task_features(int64_t n, int64_t nnz, const int64_t *csr_offsets, const int32_t *csr_nbrs,
                        void *hip_stream, float *d_feat, int64_t *ntasks_out);

/* Forward pass: d_y[m] = model(d_x[m][6]) (all device pointers). */
int triad_mlp_forward(const float *d_w, const float *d_x, int64_t m, float *d_y, void *hip_stream);

/* Mean-squared-error loss and its gradient over m samples: d_grad
 * [TRIAD_MLP_PARAMS] = d/dw (1/m) sum (model(x)-t)^2, d_loss[1] = the loss. */
int triad_mlp_loss_grad(const float *d_w, const float *d_x, const float *d_t, int64_t m, float *d_grad,
                        float *d_loss, void *hip_stream);

/* One Adam step (Kingma and Ba) on d_w with moments d_m, d_v (device,
 * TRIAD_MLP_PARAMS each) at step number t >= 1. */
int triad_mlp_adam(float *d_w, float *d_m, float *d_v, const float *d_grad, int32_t t, float lr,
                   void *hip_stream);

/* Trains the cost model on the GPU: minibatch Adam on (features, log2 cycles)
 * pairs, all device pointers; d_w holds the initial weights on entry and the
 * trained weights on return; d_loss_hist (may be NULL) receives the mean loss
 * of each epoch. */
int triad_mlp_train(float *d_w, const float *d_x, const float *d_t, int64_t m, int32_t epochs, int32_t batch,
                    float lr, uint64_t seed, void *hip_stream, float *d_loss_hist);

/* ------------------------------------------------------------------ misc */
const char *triad_last_error(void);
int triad_version(void);

/* Memory cap (process-wide; 0 = none, the default): the device memory any one
 * later call may allocate, counting its scratch (newly allocated or taken
 * from the held blocks below), the input
 * copies of triad_census / triad_census_ex and a batch plan's buffers (the
 * no-allocation census allocates nothing and is not affected). A call that
 * would go past the cap returns TRIAD_ENOMEM with nothing written to its
 * outputs. bytes < 0: TRIAD_EINVAL. Needs no device. */
int triad_set_memory_cap(int64_t bytes);

/* Held device memory. The census entry points that allocate
 * (triad_census_device, triad_labelled_census_device), triad_csr_from_arcs
 * and triad_census_update wait for their stream before they return. When the
 * stream belongs to the current device, their scratch blocks are then kept by
 * the library, per device, and reused by later calls that need a block of at
 * least the same size and at most twice it (sizes rounded up to 256 B, and to
 * whole MiB from 1 MiB on), instead of being freed and allocated again (at
 * R-MAT scale 24 a census takes about 15 GB of scratch, whose release alone
 * costs milliseconds); a stream of another device gets stream-ordered
 * allocations on that device, freed on return. At most
 * 64 GiB of free blocks are kept per device; an allocation that finds the
 * device out of memory frees that device's held blocks and tries again.
 * triad_held_memory: the bytes held now (free blocks, all devices).
 * triad_release_memory: frees every held block; returns TRIAD_OK. Blocks in
 * use by a running call are not held and are not affected. */
int64_t triad_held_memory(void);
int triad_release_memory(void);

/* Test hook for callers' error handling (not for production use): each of the
 * next `count` single-graph census calls of the process (triad_census,
 * triad_census_ex, triad_census_device, triad_census_device_noalloc,
 * triad_labelled_census_device) that gets past input validation raises the
 * device error flag after its census kernel, as a kernel that detected a
 * fault would; such a call returns TRIAD_EDEVICE and writes no output. count =
 * 0 cancels what is pending; count < 0: TRIAD_EINVAL. Needs no device. */
int triad_test_inject_device_error(int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* TRIAD_H */
