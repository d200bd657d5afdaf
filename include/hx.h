/*
 * hx.h -- C ABI of the MI355X (gfx950) halo-exchange buffer engine.
 *
 * The library implements the rank-local buffer work underneath a persistent
 * neighborhood all-to-all-v used for a sparse-matrix halo exchange, as
 * described for MPI Advance (Bienz, Schafer, Skjellum, 2023):
 *
 *   - Sec. 2.2 and Listing 4: a neighbor topology, a persistent request
 *     created once (all setup cost paid at initialisation), then driven by
 *     Start / Wait every iteration;
 *   - Sec. 2.2, last paragraph: a locality-aware variant, given unique global
 *     indices of every value exchanged, that sends a value between a pair of
 *     nodes only once and redistributes it inside the node;
 *   - Sec. 2.4: the calls accept device memory, so packing a send buffer from
 *     a vector and unpacking received data into the halo are device gathers.
 *
 * Start packs (indexed row gather from the local vector, or for the 3-step
 * variant from the rows of the rank's node); Wait runs the
 * on-node redistribution pack (locality variant) and unpacks into the halo.
 * The message transfer itself is not part of this library: a request exposes
 * its send and receive arenas, and a whole-decomposition batch ("world")
 * can simulate the transfer by copying between its ranks' arenas in the same
 * device memory.
 *
 * Conventions shared by all entry points
 *   - Every call returns an int: HX_SUCCESS (0) or a negative HX_ERR_* code.
 *     On HX_ERR_HIP, hx_last_hip_error() gives the hipError_t value.
 *     Errors are reported per calling thread (hx_last_error_message()).
 *   - Handles are opaque and returned through out-pointers; *_free(&h) sets
 *     h to NULL and accepts NULL.
 *   - "host" arrays are read during the call only and may be freed after it.
 *     "device" pointers must stay valid, unmoved and unreallocated from the
 *     call that binds them until the handle is freed (persistent semantics).
 *   - Streams are hipStream_t passed as void*; NULL means the legacy default
 *     stream.  Work is stream-ordered: a call returns once its kernels are
 *     enqueued; results are complete when the stream reaches that point.
 *   - Vectors are row-major [rows, ncols] of HX_F32 or HX_F64; one "row" is
 *     the unit every list indexes.  All index arrays are int32; every
 *     arena, halo, vector and plan must stay below 2^31 rows.
 *   - Global ownership is contiguous: rank p owns the rows/columns
 *     [row_starts[p], row_starts[p+1]).  Ranks sit on nodes of ppn ranks
 *     (the last node may be partial) as the plan's node map places them
 *     (hx_info: blocks of consecutive ranks, or round robin).
 */
#ifndef HX_H
#define HX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HX_SUCCESS = 0,
  HX_ERR_ARG = -1,         /* null handle/pointer, negative size, counts/displs inconsistent */
  HX_ERR_RANGE = -2,       /* an index outside its valid range */
  HX_ERR_STATE = -3,       /* persistent request used in the wrong state */
  HX_ERR_NOMEM = -4,       /* a device or host allocation failed */
  HX_ERR_UNSUPPORTED = -5, /* reorder != 0, sizes beyond int32 rows, unsupported variant */
  HX_ERR_HIP = -6          /* a HIP runtime call failed */
};

typedef enum { HX_F32 = 0, HX_F64 = 1 } hx_dtype;
/* Plan variants.  HX_PLAIN: one message per rank pair.  HX_LOCALITY_2STEP:
 * each rank sends its node-deduplicated data to one partner per remote node,
 * which redistributes it on its node.  HX_LOCALITY_3STEP: one message per
 * node pair, sent by the pair's aggregator A(n,m) = n*ppn + (m mod cnt(n))
 * to its receiver B(n,m) = m*ppn + (n mod cnt(m)); the aggregator packs its
 * node-mates' rows directly (node-shared memory), so its pack indices are
 * rows counted from the node's first row, and a request of such a plan reads
 * the rows of its rank's whole node (hx_req_from_plan). */
typedef enum { HX_PLAIN = 0, HX_LOCALITY_2STEP = 1, HX_LOCALITY_3STEP = 2 } hx_variant;

/* Placement of nranks ranks on NN = ceil(nranks / ppn) nodes (Sec. 2.2 groups
 * the ranks of a node without fixing which ranks share one).
 * HX_NODES_BLOCK: node(p) = p / ppn, local rank p mod ppn; the last node may
 * hold fewer ranks.  HX_NODES_CYCLIC (round robin): node(p) = p mod NN, local
 * rank p / NN.  Under either map the partner of rank q on node m is the rank
 * of node m whose local rank is lrank(q) mod (ranks on node m). */
typedef enum { HX_NODES_BLOCK = 0, HX_NODES_CYCLIC = 1 } hx_node_map;

/* Options of a plan (the info argument of a persistent init, Listing 4):
 * variant (an hx_variant); ppn >= 1 ranks per node (ignored by HX_PLAIN; a
 * value above the rank count means one node of every rank, and a plan
 * records it as the rank count);
 * node_map (an hx_node_map; the 3-step variant needs HX_NODES_BLOCK, since
 * its aggregator packs its node's rows as one contiguous range,
 * HX_ERR_UNSUPPORTED otherwise).  The fields are plain ints so that any
 * value a caller stores is checked (HX_ERR_ARG) rather than undefined. */
typedef struct {
  int variant;
  int ppn;
  int node_map;
} hx_info;

typedef struct hx_topo hx_topo;
typedef struct hx_plan hx_plan;
typedef struct hx_req hx_req;
typedef struct hx_batch hx_batch;
typedef struct hx_comm hx_comm;

/* Launch schedule of the gather / segmented-sum kernels.  A zero field means
 * "library default".  per_neighbor = 1 splits each message into its own job
 * (tiles never straddle neighbors); 0 tiles each member's rows flat. */
typedef struct {
  int tile_rows;      /* rows per tile (work unit of one workgroup iteration) */
  int block_threads;  /* 256, 512 or 1024 (the push pack runs 1024 as 512;
                         segmented sums with 1024 lanes read no LDS term
                         windows) */
  int blocks_per_cu;  /* grid = blocks_per_cu * #CUs workgroups, each walking
                         a contiguous range of tiles, but never more than
                         the tile count (rounded up to 8): a value of at
                         least tiles / #CUs (1 << 20 is the library's) gives
                         one workgroup per tile, dispatched by the hardware
                         in tile order */
  int nontemporal;    /* 1: streaming (non-temporal) loads/stores of index and
                         output (and of the terms in the chunked segmented
                         sum, and of the source rows in the push pack);
                         2: as 1, and gathers of 4- or 8-byte rows in
                         16-byte groups also stage their LDS windows with
                         streaming loads */
  int per_neighbor;   /* see above */
  int unroll;         /* rows per lane in flight: 1, 2 or 4 (0 = default);
                         with pair_rows = 1, 16-byte row groups per lane */
  int push_pack;      /* pack phase only: 1 = push form (walk the transpose of
                         the pack map, read each source row once and write it
                         to all its slots); 2 = pull form (gather per slot);
                         0 = default (push for rows of 64 bytes or more,
                         else pull) */
  int lds_window;     /* gathers: 1 = a job whose indices mostly stay inside
                         a known window of source rows (the pack: the rank's
                         own rows; the redistribution: its stage-1 receive
                         arena; a world's unpack: its stage-2 receive arena)
                         copies that window into LDS (when it fits in 80 KiB
                         and holds at least half of the job's indices,
                         counted on the device when the launch table is
                         built) and gathers rows inside it from LDS, the
                         others from global memory; 2 = gather from global
                         memory; 0 = default (1 for rows of 16 bytes or
                         less, else 2) */
  int pair_rows;      /* gathers of 4- or 8-byte rows: 1 = 16 bytes of rows
                         per lane (a group of four or two consecutive rows
                         takes one vector load of its indices and one
                         16-byte store; with LDS windows the window is
                         staged while the tile's indices are in flight),
                         taken where every job's index list is congruent
                         with its destination (one first row aligns both);
                         2 = one row per lane; 0 = default (1 for rows of
                         4 or 8 bytes, with 16384-row tiles, 512 lanes, one
                         workgroup per tile and 4 groups per lane) */
} hx_sched;

/* ---------------------------------------------------------------------------
 * Errors
 * ------------------------------------------------------------------------- */
const char* hx_error_string(int code);
int hx_last_hip_error(void);
const char* hx_last_error_message(void);
/* Library version string (build identifier). */
const char* hx_version(void);

/* ---------------------------------------------------------------------------
 * Device memory allocator -- Sec. 2.4 (the library works on device memory
 * of the caller's memory space).
 *
 * Every device allocation the library makes (plan arrays, send / receive
 * arenas, launch tables, temporaries of the plan build) goes through
 * alloc_fn(bytes, stream, ctx), where stream is the hipStream_t the memory
 * is first used on (NULL when the call has none: the legacy default
 * stream), and is returned through free_fn(ptr, ctx).  alloc_fn returns
 * device memory of the current device, aligned to at least 16 bytes, or
 * NULL on failure; the library then fails the call with HX_ERR_NOMEM and
 * frees whatever that call had already allocated (no leak).  A pointer
 * that is not 16-byte aligned is returned at once through free_fn and the
 * call fails with HX_ERR_ARG.  Before free_fn runs the library waits for
 * the device to be idle (as hipFree does), so the allocator may hand the
 * block out again at once.
 * hx_set_allocator(NULL, NULL, NULL) restores hipMalloc / hipFree.  The
 * setting is process-wide and applies to allocations made after the call;
 * each block is freed through the free_fn that was installed when it was
 * allocated, so alloc_fn, free_fn and ctx must stay valid until every
 * handle allocated under them is freed.  Exactly one of the two functions
 * NULL: HX_ERR_ARG.  The Python binding installs torch's caching allocator
 * (torch.cuda.caching_allocator_alloc / _delete), so torch sees and reuses
 * the library's memory.
 * ------------------------------------------------------------------------- */
typedef void* (*hx_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*hx_free_fn)(void* ptr, void* ctx);
int hx_set_allocator(hx_alloc_fn alloc_fn, hx_free_fn free_fn, void* ctx);

/* ---------------------------------------------------------------------------
 * Neighbor topology -- Listing 4 (MPIX_Dist_graph_create_adjacent).
 *
 * rank, nranks: this rank and the size of the (simulated) communicator.
 * recv_procs[n_recvs], send_procs[n_sends] (host): distinct neighbor ranks in
 * [0, nranks), none equal to rank.  Weights are accepted and ignored (may be
 * NULL).  reorder must be 0 (HX_ERR_UNSUPPORTED otherwise), since ranks are
 * fixed by the decomposition.  HX_ERR_RANGE on an out-of-range or duplicate
 * neighbor.  The handle owns host copies of the lists.
 * ------------------------------------------------------------------------- */
int hx_topo_create(int rank, int nranks, int n_recvs, const int* recv_procs,
                   const int* recv_weights, int n_sends, const int* send_procs,
                   const int* send_weights, int reorder, hx_topo** out);
int hx_topo_free(hx_topo** topo);

/* ---------------------------------------------------------------------------
 * Persistent plain request -- Listing 4 (MPIX_Neighbor_alltoallv_init).
 *
 * x_local   device [n_local, ncols]: the vector the send buffer is packed from.
 * sendcounts, sdispls (host [n_sends]): all-to-all-v layout of the send arena;
 *           sdispls may be NULL, otherwise it must equal the exclusive prefix
 *           sum of sendcounts (the arena is packed densely, neighbor order).
 * send_idx  host [sum(sendcounts)]: the local row of x_local copied into each
 *           send slot (the pack map), each in [0, n_local).
 * halo      device [sum(recvcounts), ncols]: receives the unpacked values in
 *           neighbor order (the plain unpack is the identity copy of the
 *           receive arena into the halo).
 * recvcounts, rdispls (host [n_recvs]): as for the send side.
 * The library allocates and owns the send and receive arenas
 * (hx_req_arena) and the device copies of all lists, and builds the
 * transpose of the pack map (rows -> send slots, ascending) for hx_backward.
 * Errors: HX_ERR_ARG (nulls, counts < 0, displs not the prefix sum),
 * HX_ERR_RANGE (send_idx out of range), HX_ERR_UNSUPPORTED (>= 2^31 rows).
 * ------------------------------------------------------------------------- */
int hx_neighbor_alltoallv_init(const void* x_local, int64_t n_local,
                               const int* sendcounts, const int* sdispls, const int* send_idx,
                               void* halo, const int* recvcounts, const int* rdispls,
                               hx_dtype dtype, int ncols, const hx_topo* topo, hx_req** out);

/* ---------------------------------------------------------------------------
 * Per-rank locality-aware init -- Sec. 2.2, last paragraph (the extension
 * takes, beside the neighbor lists, the global indices of all values sent
 * and received).  Deduplicating over a node needs what every rank of the
 * node receives, so the init is collective over a communicator; one process
 * plays every rank of a simulated one:
 *
 * hx_comm_create: nranks ranks owning rows [row_starts[r], row_starts[r+1])
 *   (host [nranks+1], copied), info (host, copied; any variant, the 3-step
 *   one with HX_NODES_BLOCK only, else HX_ERR_UNSUPPORTED), stream: where
 *   the plan is built when the set completes.
 * hx_neighbor_locality_alltoallv_init: rank topo->rank joins.  Arguments as
 *   for hx_neighbor_alltoallv_init (displacements NULL or the prefix sums),
 *   with global indices instead of local rows: global_sindices host
 *   [sum(sendcounts)] int64, each owned by this rank; global_rindices host
 *   [sum(recvcounts)] int64, the message from recv_procs[i] holding indices
 *   owned by that rank, distinct over the whole receive list, in any order
 *   (halo row u receives global index global_rindices[u]).  n_local must be
 *   the rank's row count; for the 3-step variant x_local is instead the
 *   first row of the rank's node in node-shared memory and n_local the
 *   node's row count, as for hx_req_from_plan (send indices stay the rank's
 *   own rows).  Lists are copied.  Until every rank has joined
 *   the returned request is pending: every call on it but hx_req_free
 *   returns HX_ERR_STATE.  The call that completes the set checks that what
 *   q sends to s is, element for element, what s receives from q, builds the
 *   plan on the GPU from the receive indices (hx_plan_from_halos) and fills
 *   every joined request; its Start/Wait then run the plan's stages and the
 *   unpack writes each halo row in the caller's receive order.  Errors of the
 *   completing call (HX_ERR_ARG for lists that do not match) are returned by
 *   it, without a request; the set's other requests then stay pending.
 *   HX_ERR_STATE for a rank that joins twice or a set that is over.
 * hx_comm_free: may be called at any time; requests of an incomplete set
 *   stay pending, completed requests are independent of the communicator.
 * ------------------------------------------------------------------------- */
int hx_comm_create(int nranks, const int64_t* row_starts, const hx_info* info, void* stream, hx_comm** out);
int hx_neighbor_locality_alltoallv_init(const void* x_local, int64_t n_local, const int* sendcounts,
                                        const int* sdispls, const int64_t* global_sindices, void* halo,
                                        const int* recvcounts, const int* rdispls,
                                        const int64_t* global_rindices, hx_dtype dtype, int ncols,
                                        const hx_topo* topo, hx_comm* comm, hx_req** out);
int hx_comm_free(hx_comm** comm);

/* ---------------------------------------------------------------------------
 * Plans of a whole decomposition, built on the GPU (all setup at init,
 * Sec. 2.2), for the plain variant or the locality-aware variants.  This is
 * the collective half of the locality-aware init: every rank's halo goes in
 * at once, since deduplication over a node and the partner assignment need
 * the halos of all ranks; hx_req_from_plan then gives one rank its request
 * (the per-rank half).
 *
 * hx_plan_from_csr: halo discovery from the sparse structure, then as below.
 *   row_starts host [nranks+1] int64, increasing, row_starts[0] = 0, n = row_starts[nranks];
 *   row_ptr    device [n+1] int64 (CSR row pointers);
 *   cols       device [row_ptr[n]] int32, each in [0, n).
 * hx_plan_from_halos: the locality-aware extension's input (Sec. 2.2, last
 *   paragraph): the unique global indices every rank receives.
 *   halo_ptr   host [nranks+1] int64; halo_cols device [halo_ptr[nranks]] int32,
 *   strictly increasing within each rank and never owned by that rank.
 * For each rank the plan holds (the lists a persistent init would build):
 *   halo, stage-1 send/recv lists (plain: all messages; locality: on-node
 *   messages plus one deduplicated message per remote node, sent to the
 *   partner there), stage-2 (redistribution) lists,
 *   the unpack map into the halo, and the transpose of the pack map.
 * hx_plan_from_csr marks one bit per (rank, column) to find the halos; it
 * does so for a group of ranks at a time, holding at most 1 GiB of bitmaps
 * (the environment variable HX_PLAN_BITMAP_BYTES, read at each call, sets
 * another budget; a group has at least one rank).
 * info (host, read during the call): variant, ranks per node and node map.
 * The plan owns its device arrays; inputs are read during the call only.
 * The call synchronises stream before returning.  Errors: HX_ERR_ARG (null
 * info, ppn < 1, unknown variant or node map), HX_ERR_RANGE (column out of
 * range, halo not strictly increasing or owned by its rank),
 * HX_ERR_UNSUPPORTED (sizes beyond int32, the dense rank-pair tables
 * exceeding HX_PLAN_MAX_RANKS ranks, the 3-step variant with a cyclic map).
 * ------------------------------------------------------------------------- */
#define HX_PLAN_MAX_RANKS 16384
int hx_plan_from_csr(int nranks, const int64_t* row_starts, const hx_info* info,
                     const int64_t* row_ptr, const int32_t* cols, void* stream, hx_plan** out);
int hx_plan_from_halos(int nranks, const int64_t* row_starts, const hx_info* info,
                       const int64_t* halo_ptr, const int32_t* halo_cols, void* stream,
                       hx_plan** out);
int hx_plan_free(hx_plan** plan);

/* Per-rank plan arrays, copied to host memory.  Field ids and element counts
 * (all int32): */
typedef enum {
  HX_F_HALO = 0,      /* [H]        global column ids of the halo, ascending */
  HX_F_S1_PROCS,      /* [n_s1]     stage-1 destinations, ascending */
  HX_F_S1_COUNTS,     /* [n_s1] */
  HX_F_S1_DISPLS,     /* [n_s1]     exclusive prefix of counts */
  HX_F_S1_IDX,        /* [E1]       local row packed into each stage-1 send slot (3-step:
                                      row counted from the node's first row) */
  HX_F_R1_PROCS,      /* [n_r1]     stage-1 sources, ascending */
  HX_F_R1_COUNTS,     /* [n_r1] */
  HX_F_R1_DISPLS,     /* [n_r1] */
  HX_F_S2_PROCS,      /* [n_s2]     redistribution destinations (same node) */
  HX_F_S2_COUNTS,     /* [n_s2] */
  HX_F_S2_DISPLS,     /* [n_s2] */
  HX_F_S2_SRC,        /* [E2]       stage-1 receive slot forwarded by each stage-2 send slot */
  HX_F_R2_PROCS,      /* [n_r2] */
  HX_F_R2_COUNTS,     /* [n_r2] */
  HX_F_R2_DISPLS,     /* [n_r2] */
  HX_F_UNPACK_SRC,    /* [H]        slot of halo entry j in [stage-1 recv | stage-2 recv] */
  HX_F_BT_PTR,        /* [n_local+1] transpose of the pack map: row -> slots (3-step: over
                                      the node's rows) */
  HX_F_BT_PERM,       /* [E1]       send slots grouped by local row, ascending */
  HX_F_COUNT
} hx_field;
/* Number of int32 elements of a field for a rank (HX_ERR_RANGE for a bad rank/field). */
int hx_plan_field_size(const hx_plan* plan, int rank, hx_field field, int64_t* count);
/* Copies a field to host memory dst (capacity given by hx_plan_field_size). */
int hx_plan_field_copy(const hx_plan* plan, int rank, hx_field field, int32_t* dst);
/* A field of every rank at once (host memory): offsets [nranks+1] (may be
 * NULL) receives where each rank's array starts in the concatenation in rank
 * order, dst (capacity offsets[nranks] elements; may be NULL) the
 * concatenation.  Synchronous. */
int hx_plan_field_all(const hx_plan* plan, hx_field field, int64_t* offsets, int32_t* dst);
/* What a plan was built from: its rank count, rows n, info, and (row_starts
 * non-NULL, capacity nranks+1) its row starts.  Any output may be NULL.
 * With the halo field this is all a plan needs to be built again
 * (hx_plan_from_halos gives the same arrays: plan building is deterministic),
 * which is how a plan is saved and restored. */
int hx_plan_describe(const hx_plan* plan, int* nranks, int64_t* n, hx_info* info, int64_t* row_starts);

/* Persistent request for one rank of a plan (its arrays stay on the device).
 * x_local device [n_local, ncols]: the rank's own rows (n_local of them);
 * halo device [H, ncols].  For a 3-step plan x_local is instead the first row
 * of the rank's node in memory the node's ranks share, and n_local the
 * node's row count: an aggregator packs its node-mates' rows (the on-node
 * gather of the 3-step scheme).  The backward of such a request then writes
 * g_x [n_local, ncols] over the node's rows too: this request's share of
 * their gradient (the sums over its own send slots; rows it never packs get
 * +0.0), which the node's ranks add up.  HX_ERR_ARG, HX_ERR_RANGE (a plan
 * whose arrays are inconsistent), HX_ERR_NOMEM, HX_ERR_HIP. */
int hx_req_from_plan(const hx_plan* plan, int rank, const void* x_local, void* halo,
                     hx_dtype dtype, int ncols, hx_req** out);

/* ---------------------------------------------------------------------------
 * Start / Wait -- Listing 4 (MPIX_Start, MPIX_Wait).
 *
 * hx_start: pack the stage-1 send arena from x_local (inactive -> active;
 *   HX_ERR_STATE if already active).
 * hx_wait: redistribution pack (locality variant) from the receive arena,
 *   then unpack into the halo (active -> inactive).  Waiting on an inactive
 *   request returns HX_SUCCESS and does nothing, as for an inactive
 *   persistent MPI request.  Both calls only enqueue work on stream.
 * The receive arena is filled by the (not built) transport between Start and
 * Wait; callers simulate it by writing into hx_req_arena(HX_ARENA_RECV).
 * ------------------------------------------------------------------------- */
int hx_start(hx_req* req, void* stream);
int hx_wait(hx_req* req, void* stream);

enum { HX_ARENA_SEND = 0, HX_ARENA_RECV = 1, HX_ARENA_GRAD_SEND = 4 };
/* Device pointer and row count of a request's arena.  Send arena layout:
 * [stage-1 send (E1) | stage-2 send (E2)]; receive arena:
 * [stage-1 recv (R1) | stage-2 recv (R2)]; rows of ncols values. */
int hx_req_arena(hx_req* req, int which, void** dev_ptr, int64_t* rows);

/* Backward of the pack (the differentiable path): for every local row i,
 * g_x[i] = sum over stage-1 send slots k packed from row i, in ascending k, of
 * g_send[k]; adds only, in the request's dtype, first term first (a lone
 * -0.0 stays -0.0), rows never packed get +0.0.  g_send device [E1, ncols],
 * g_x device [n_local, ncols]; bound persistently. */
int hx_req_bind_grad(hx_req* req, const void* g_send, void* g_x);
/* Partition-ready pack: the GPU half of partitioned, early-bird sends
 * (Sec. 2.3: portions of a buffer marked ready may leave before the whole
 * message is complete; here each stage-1 message is one partition).
 * hx_req_enable_ready allocates one 64-bit completion counter per stage-1
 * message (in the order of the request's send list), zeroed, owned by the
 * request, and returns their device address.  From then on the pack runs in
 * the pull form with one job per message, and after each tile the rows it
 * wrote are added to its message's counter once they are visible
 * device-wide (release fence, then atomic add).  After the k-th pack since
 * enabling (hx_start, a batch Start, or hx_batch_launch_phase of the pack;
 * the tuner's trial launches do not count), counter[m] reaches
 * k * sendcounts[m] exactly when message m of that pack is complete, so a
 * transport (a kernel on another stream, a copy engine) may send each
 * message as soon as its counter reaches the target (with an acquire load)
 * instead of waiting for the whole pack.  Counters only grow (nothing to
 * reset inside captured graphs).  Batches take the mode from their members
 * at hx_batch_init (their pack then runs in the pull form).  HX_ERR_STATE
 * while the request is active. */
int hx_req_enable_ready(hx_req* req, unsigned long long** dev_counters);
int hx_backward(hx_req* req, void* stream);

/* ---------------------------------------------------------------------------
 * Backward that allocates nothing.  For callers that cannot allocate device
 * memory during the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.
 *
 * Computes what hx_req_bind_grad(req, g_send, g_x) followed by
 * hx_backward(req, stream) computes, bit for bit: for every local row i,
 * g_x[i] = sum over the stage-1 send slots k packed from row i, ascending k,
 * of g_send[k] (first term first, +0.0 for rows never packed).  g_send
 * device [E1, ncols] (may be NULL when E1 = 0), g_x device [n_local, ncols],
 * both in the request's dtype; they are used by this call only and the
 * request's bound gradients are left as they are.
 * The segmented sum's launch table (job descriptor, tile prefix and each
 * tile's entry range) is written by a kernel on stream into a fixed
 * library-owned device area of HX_NOALLOC_SCRATCH_BYTES per GPU, held from
 * the first call on that GPU until the process ends, instead of device
 * memory allocated for the request: the call makes no allocation (neither
 * hipMalloc nor the installed allocator) and no memset, only two kernel
 * launches on stream.
 * Limit: the sum's tiles, ceil(n_local / tile_rows) with tile_rows between
 * 64 and 512 chosen from the row size (512 for rows of 128 bytes or less),
 * must fit the area: at most (HX_NOALLOC_SCRATCH_BYTES - 512) / 8 = 131008
 * tiles; beyond that the call fails with HX_ERR_UNSUPPORTED and launches
 * nothing.
 * Every call on a GPU uses that GPU's one area: calls issued in order on one
 * stream are safe, calls that overlap on one GPU (other streams, or threads
 * without ordering) race and give wrong results.
 * Errors: HX_ERR_ARG (null request, null g_send with E1 > 0, null g_x with
 * n_local > 0), HX_ERR_UNSUPPORTED, HX_ERR_HIP.
 * ------------------------------------------------------------------------- */
#define HX_NOALLOC_SCRATCH_BYTES (1u << 20)
int hx_backward_noalloc(hx_req* req, const void* g_send, void* g_x, void* stream);
/* Frees a request (NULL or *req NULL: nothing).  HX_ERR_STATE, and nothing
 * freed, while the request is active (Start without Wait) or a member of a
 * batch that has not been freed. */
int hx_req_free(hx_req** req);

/* ---------------------------------------------------------------------------
 * Batches: many persistent requests driven as one (one multi-job kernel per
 * phase, captured in a hipGraph at init and replayed by start/wait).
 *
 * hx_batch_init: members are existing requests (same dtype and ncols); they
 *   stay owned by the caller and must outlive the batch.  sched NULL = use a
 *   cached tuned schedule for this shape if one exists, else the default.
 * hx_batch_from_plan: every rank of a plan as one batch over flat arrays
 *   ("world").  x_global device [n, ncols]; halo_all device [sum H, ncols]
 *   (ranks in order).  With flags & HX_WORLD_SIM_TRANSFER, start also copies
 *   each stage-1 message into its receiver's arena and wait copies each
 *   stage-2 message likewise (the simulated transport; not part of the
 *   path's own work).  The world's backward is the full adjoint of the
 *   exchange: g_x[c] = sum over ranks s (ascending) whose halo holds c of
 *   g_halo_all at that entry, fixed order as hx_backward.  With flags &
 *   HX_WORLD_STAGED_BACKWARD a locality plan's backward instead runs the
 *   forward's stages in reverse, each rank-local (same value in exact
 *   arithmetic, another grouping of the sums): the reverse unpack scatters
 *   g_halo_all into the receive slots; the stage-2 messages travel back;
 *   each forwarder sums per stage-1 receive slot its own halo's term, then
 *   its redistribution entries in ascending entry (= destination rank); the
 *   stage-1 messages travel back; each owner sums its send slots per row in
 *   ascending slot.  The two travels are the simulated transport (run with
 *   HX_WORLD_SIM_TRANSFER).  Plain plans: the flag changes nothing (their
 *   backward is already the owner sums after the reverse stage-1 travel).
 * hx_batch_start / hx_batch_wait: Start / Wait of all members (graph launch).
 * hx_batch_start_plain / hx_batch_wait_plain: the same work as one launch per
 *   member (the plain one-plan-per-launch form, for comparison).
 * hx_batch_tune: times candidate schedules on the batch's own buffers (the
 *   candidates write the same arenas/halos a start/wait would), keeps the
 *   fastest, re-captures the graphs, and records it in the tuning cache
 *   (file named by HX_TUNE_CACHE, if set).  Search per phase: tile size x
 *   rows per lane x pack form x LDS windows x rows per lane pairing (8-byte
 *   rows), then launch shape (persistent or one-shot grid, workgroup size) x
 *   streaming hints, then the first dimensions again, then rows per lane x
 *   launch shape together; each candidate is the average of three
 *   back-to-back launches (short kernels: about a millisecond of launches,
 *   at most 50), best of two trials.  Then the
 *   replay (see hx_batch_set_replay): graph or direct launches, whichever
 *   runs 20 start + wait steps faster.  With HX_TUNE_LOG set, every
 *   candidate's time goes to stderr.
 * ------------------------------------------------------------------------- */
enum { HX_WORLD_SIM_TRANSFER = 1, HX_WORLD_STAGED_BACKWARD = 2 };
int hx_batch_init(hx_req* const* reqs, int n, const hx_sched* sched, hx_batch** out);
int hx_batch_from_plan(const hx_plan* plan, const void* x_global, void* halo_all,
                       hx_dtype dtype, int ncols, int flags, const hx_sched* sched,
                       hx_batch** out);
int hx_batch_start(hx_batch* b, void* stream);
int hx_batch_wait(hx_batch* b, void* stream);
int hx_batch_start_plain(hx_batch* b, void* stream);
int hx_batch_wait_plain(hx_batch* b, void* stream);
/* Backward: member batches use each member's bound gradients; worlds use
 * g_in = g_halo_all [sum H, ncols] and g_out = g_x_global [n, ncols]. */
int hx_batch_bind_grad(hx_batch* b, const void* g_in, void* g_out);
int hx_batch_backward(hx_batch* b, void* stream);
int hx_batch_backward_plain(hx_batch* b, void* stream);
int hx_batch_tune(hx_batch* b, void* stream);
/* hx_batch_launch_phase: launch the kernel of one phase alone
 *   (0 pack, 1 redistribution, 2 unpack, 3 backward) from the same launch
 *   table the graphs replay, outside the Start/Wait state machine, so that a
 *   caller can time each kernel; the simulated transfers are not run.
 *   HX_ERR_STATE while a Start is pending, or for the backward before
 *   gradients are bound (members: before the first hx_batch_backward after
 *   binding). */
int hx_batch_launch_phase(hx_batch* b, int phase, void* stream);
/* The schedule in use for a phase (0 pack, 1 redistribution, 2 unpack, 3 backward). */
int hx_batch_get_sched(const hx_batch* b, int phase, hx_sched* out);
/* Sets the schedule of one phase (zero fields: library defaults, as for
 * hx_batch_init) and rebuilds the launch tables and graphs, so that a
 * schedule recorded with hx_batch_get_sched (or tuned elsewhere) can be
 * applied without tuning; the tuning cache is not written.  HX_ERR_ARG
 * (null, bad phase, an invalid schedule: the batch then keeps its previous
 * one), HX_ERR_STATE while a Start is pending. */
int hx_batch_set_sched(hx_batch* b, int phase, const hx_sched* sched);
/* Replay of start / wait / backward: HX_REPLAY_GRAPH (default) launches the
 * graph captured at init; HX_REPLAY_DIRECT launches the same prepared launch
 * tables one by one (no per-call setup either way, same results).  A graph
 * launch has a fixed cost (about 15 us measured on MI355X, whatever the
 * graph holds) against about 3 us per directly launched kernel, so steps of
 * a few short kernels replay faster directly; hx_batch_tune measures a
 * start + wait both ways and keeps the faster.  Mode other than these two:
 * HX_ERR_ARG. */
enum { HX_REPLAY_GRAPH = 0, HX_REPLAY_DIRECT = 1 };
int hx_batch_set_replay(hx_batch* b, int mode);
int hx_batch_get_replay(const hx_batch* b, int* mode);
/* World arenas: which = HX_ARENA_SEND / HX_ARENA_RECV, all ranks concatenated
 * as [stage-1 part of every rank | stage-2 part of every rank].
 * which = HX_ARENA_GRAD_SEND (plain or staged-backward worlds, after
 * hx_batch_bind_grad): the gradient slots of every rank's stage-1 send arena,
 * laid out as the send arena's stage-1 part.  The world backward sums these
 * slots per owned row; with HX_WORLD_SIM_TRANSFER the library fills them
 * (the reverse transfer), otherwise the caller's transport must.  Locality
 * worlds without the staged backward read g_halo_all directly.
 * hx_batch_arena_offset gives the first row of a rank's stage-1 part
 * (which = HX_ARENA_SEND / HX_ARENA_RECV) or stage-2 part (which | 2);
 * rank = nranks gives the end of the part. */
int hx_batch_arena(hx_batch* b, int which, void** dev_ptr, int64_t* rows);
int hx_batch_arena_offset(hx_batch* b, int which, int rank, int64_t* row_offset);
/* Algorithmic bytes moved per phase launch (phase as in hx_batch_get_sched):
 * each read of a distinct source row, each output row written, each index
 * (phase 3 of a staged locality world: forwarder sums + owner sums). */
int hx_batch_bytes(const hx_batch* b, int phase, int64_t* bytes);
int hx_batch_free(hx_batch** b);

#ifdef __cplusplus
}
#endif
#endif /* HX_H */
