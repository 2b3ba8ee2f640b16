/*
 * gheap.h -- C ABI of libgheap.so, a generalized concurrent min-heap for
 * AMD Instinct MI355X (gfx950).
 *
 * The heap is the generalized heap of Chen et al., "Accelerating Concurrent
 * Heap on GPUs" (Sec. 3): every node holds a sorted batch of k entries, a
 * partial buffer holds fewer than k entries that are all >= the root's
 * (Sec. 3.1, Properties 1-3), deleteMin returns the root batch, and insert
 * and deleteMin run top-down under per-node locks with many operations in
 * flight (Sec. 3.3, TD-INS/TD-DEL heap).
 *
 * Entries.  A heap set has one key type, fixed at creation:
 *   GH_U32_ID  8-byte entries, an unsigned 64-bit integer ordered as an
 *              integer; (key, id) pairs are packed by the caller as
 *              (uint64_t)key << 32 | id;
 *   GH_I64_ID  16-byte entries, two 64-bit words ordered lexicographically,
 *              the word at the lower address first: a signed 64-bit key
 *              stored biased (key XOR 2^63, so that it orders as unsigned),
 *              then a 32-bit id and 32 zero bits (the second word is
 *              id | 0 << 32 on a little-endian device).
 * Every buffer of entries (d_keys, d_sorted, d_in, d_out, ...) holds entries
 * of the set's width, and entry offsets and counts are in entries.  The
 * all-ones entry of either width is reserved as the empty-slot filler and
 * must never be inserted (an id of 0xFFFFFFFF never forms it with a real
 * key).  Equal entries are indistinguishable, so results are unique even
 * with repeated keys.
 *
 * Memory and streams.  Every pointer named d_* is a device pointer on the
 * current HIP device.  The caller owns all device buffers, including the
 * arena that holds the heap state (size from heap_arena_bytes); the library
 * owns only the handle.  All calls are ordered on the stream given at
 * creation (a hipStream_t passed as void*, NULL = the legacy default stream)
 * and return before the device work finishes, except where noted.  Input
 * buffers must stay valid and unmodified, and output buffers untouched, until
 * the stream has passed the call.  A handle must not be used from two host
 * threads at once.
 *
 * Errors.  Functions return GH_OK (0) or a negative GH_E* code.  Argument
 * errors are reported synchronously and leave the heap unchanged.  Errors
 * found on the device (capacity exceeded inside a multi-op submission, a
 * lock wait over the watchdog limit) are sticky: they are reported by
 * heap_sync, heap_size and heap_destroy, and every later operation on the
 * handle returns the same code.
 *
 * Linearization.  Every operation takes a ticket when it acquires the root;
 * the root is the linearization point of the TD-INS/TD-DEL heap (Sec. 3.3.3,
 * Theorem 1), so applying the operations one at a time in ticket order on a
 * sequential generalized heap reproduces every deleteMin result exactly.
 * Within one heap, tickets follow submission order.
 */
#ifndef GHEAP_H
#define GHEAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GH_OK 0
#define GH_EINVAL (-1)     /* bad argument: null pointer, unsupported k, ... */
#define GH_ENOMEM (-2)     /* arena too small, or an insert exceeds capacity */
#define GH_ETIMEDOUT (-3)  /* a device lock wait exceeded the watchdog limit */
#define GH_EDEVICE (-4)    /* a HIP runtime call failed */
#define GH_ESTATE (-5)     /* the heap set was left inconsistent by an earlier error */

#define GH_OP_INSERT 0u
#define GH_OP_DELETE_MIN 1u

/* Key types (entry layouts) of a heap set; see "Entries" above. */
#define GH_U32_ID 0   /* 8 bytes: u32 key above u32 id */
#define GH_I64_ID 1   /* 16 bytes: biased i64 key, then u32 id and u32 zero */

/* Opaque handle to a set of one or more heaps that share k, an arena and a
 * stream.  heap_create makes a set of one heap. */
typedef struct gh_heap *gh_heap_t;

/* One operation of a multi-operation submission (32 bytes, device memory).
 *   heap   index of the heap within the set, < nheaps
 *   kind   GH_OP_INSERT or GH_OP_DELETE_MIN
 *   n      insert: number of entries, 1..k, or with GH_TUNE_MULTI_INSERT
 *          1..heap_insert_max(k) (an insert of more than k entries takes the
 *          root once: see heap_insert_max); deleteMin: number of entries to
 *          take, 1..k, 0 meaning k (a deleteMin of c < k entries returns
 *          the min(c, size) smallest; heap_submit runs those only with
 *          GH_TUNE_VARIABLE_DELETE); larger n is rejected (GH_EINVAL)
 *   seq    rank of this operation among the submission's operations on the
 *          same heap: 0, 1, 2, ... in the order they must take the root
 *   off    insert: entry offset of its keys in d_in; deleteMin: entry offset
 *          of its output slot in d_out (room for its count of entries)
 *   arrival_ns  earliest start, in nanoseconds after the submission starts
 *          on the device (0 = immediately); operations must appear in
 *          non-decreasing arrival order */
typedef struct gh_op {
    uint32_t heap;
    uint32_t kind;
    uint32_t n;
    uint32_t seq;
    uint64_t off;
    uint64_t arrival_ns;
} gh_op;

/* Per-operation record written by a submission (32 bytes, device memory).
 *   ticket   root ticket of the operation on its heap (linearization order)
 *   count    insert: n; deleteMin: entries returned (min(c, heap size) for a
 *            deleteMin of c entries)
 *   levels   insert: depth of the target node reached (0 if the keys stayed
 *            in the partial buffer; the deepest target of an insert of more
 *            than k entries); deleteMin: sift-down levels that merged
 *   kind     GH_OP_INSERT or GH_OP_DELETE_MIN
 *   flags    bit 0: a full batch was created; bit 1: an insert handed its
 *            batch to a deleteMin that took its target; bit 2: a deleteMin
 *            took the batch of an in-flight insert; bit 3: the heap had at
 *            least one node when the root was taken; bit 4: a deleteMin
 *            refilled the root from the last node; bit 5: a bottom-up
 *            insert's climb stopped below the root (GH_TUNE_BOTTOM_UP);
 *            bit 6: the operation was rejected (capacity or malformed
 *            record); bit 7: abandoned after a device error
 *   pb       partial-buffer size when the root was taken
 *   t_claim, t_root, t_done  device wall clock in ticks (heap_clock_hz)
 *            relative to the submission's start, when a workgroup claimed
 *            the operation, took the root, and finished (32-bit, wraps) */
typedef struct gh_logrec {
    uint64_t ticket;
    uint32_t count;
    uint16_t levels;
    uint8_t kind;
    uint8_t flags;
    uint16_t pb;
    uint16_t reserved;
    uint32_t t_claim;
    uint32_t t_root;
    uint32_t t_done;
} gh_logrec;

/* Per-request record written by heap_serve (32 bytes, device memory).
 *   first_ticket  root ticket of the request's first operation on its heap
 *   count         deleteMin: entries returned; insert: entries inserted
 *                 (0 if rejected)
 *   nops          operations the request was split into (ceil(n /
 *                 heap_insert_max(k)) for an insert, 1 for a deleteMin)
 *   kind          GH_OP_INSERT or GH_OP_DELETE_MIN
 *   flags         bit 0: admitted; bit 1: an insert waited for heap memory;
 *                 bit 6: rejected (larger than the heap's capacity, never
 *                 fitted before the stream ended, or a malformed record)
 *   t_admit, t_resp, t_done  device wall clock in ticks after the start of
 *                 the serving launch (32-bit): admission; the answer (the
 *                 last operation released the root: a deleteMin's entries
 *                 are in d_out, an insert's entries are seen by every later
 *                 operation on the heap); completion of the last operation
 *                 (the node updates below the root that follow the answer
 *                 are done)
 *   bytes         algorithmic bytes of the request's operations: what the
 *                 method moves between HBM and the workgroups along the
 *                 paths the operations took (node loads and stores, partial
 *                 buffer, input and output), entry bytes e, node capacity k,
 *                 n entries, s partial-buffer entries, L levels merged: an
 *                 insert into the partial buffer 2e(n + s) (+ 2ek with a
 *                 root), a full batch e(n + s + (n + s - k)) + e(2kL + k); a
 *                 deleteMin 2es with no node, 2ek from the root alone,
 *                 ek(3 + 4L) + 2es refilled from the last node */
typedef struct gh_reqrec {
    uint64_t first_ticket;
    uint32_t count;
    uint16_t nops;
    uint8_t kind;
    uint8_t flags;
    uint32_t t_admit;
    uint32_t t_done;
    uint32_t t_resp;
    uint32_t bytes;
} gh_reqrec;

/* Launch shape of a submission: workgroups = number of operations in flight
 * (0 = library default), threads = workgroup size (0 = library default: 64
 * for k = 32, 128 for k = 64 and 128, 512 for k = 256 and 512, 1024 for
 * k = 1024; heap_serve: 256 for k >= 256; must be one of the shapes
 * heap_supported_shape accepts for k).  flags: 0, or any of
 * GH_TUNE_VARIABLE_DELETE when the submission holds deleteMins of fewer than
 * k entries and GH_TUNE_MULTI_INSERT when it holds inserts of more than k
 * entries; such submissions run in a general kernel of their own, so that
 * submissions of whole-root deleteMins and inserts of up to k entries keep a
 * kernel compiled without those code paths.  Without the flag such a record
 * is rejected (GH_EINVAL). */
#define GH_TUNE_VARIABLE_DELETE 1u
#define GH_TUNE_MULTI_INSERT 2u
/* GH_TUNE_BOTTOM_UP: run the submission's inserts bottom-up (Sec. 3.2.2,
 * "Bottom-up INS" paragraph; the BU-INS of Sec. 3.3.4), for insert phases:
 * every operation must be an insert of 1..k entries; a deleteMin record is
 * rejected (GH_EINVAL), and the flag may not be combined with the two above
 * (GH_EINVAL, nothing runs).  Each insert takes the root in ticket order
 * only to merge its batch with the partial buffer (and, if everything fits
 * there, the partial buffer with the root, as the top-down insert does);
 * a full batch of k entries goes to its target node and climbs, merging
 * with each parent (the parent keeping the k smallest) until the parent's
 * largest entry is no larger than the batch's smallest or the root is
 * merged.  One operation at a time this leaves exactly the top-down
 * layout; with many in flight the heap satisfies Properties 1-3 with the
 * same entries when the launch ends, and its layout may differ.  Inserts
 * do not overlap deleteMins in this form because a climbing insert has no
 * linearization point that deleteMins in flight would respect (a deleteMin
 * can pass a climbing batch and miss entries smaller than the ones it
 * returns); deleteMins run in other submissions.  Log records: levels =
 * merges of the climb; flags bit 5 = the climb stopped below the root. */
#define GH_TUNE_BOTTOM_UP 4u
/* GH_TUNE_SHARED_ROOT: a submission of whole-root operations (no other
 * flag) launched with one workgroup runs the per-operation root protocol
 * (ticket and node locks) like any other launch.  Without the flag such a
 * submission runs with one operation in flight and no locks: each heap's root
 * and partial buffer stay in the workgroup's LDS while its operations run,
 * in list order, and its nodes are reached with caching loads and stores.
 * The results and the heap layout are the same; a record whose seq is not
 * its heap's next (one workgroup takes the root in list order) is refused
 * (GH_EINVAL) instead of waiting. */
#define GH_TUNE_SHARED_ROOT 8u
typedef struct gh_tuning {
    uint32_t workgroups;
    uint32_t threads;
    uint32_t flags;
} gh_tuning;

/* Bytes of arena needed for nheaps heaps of node capacity k and key type
 * keytype, heap i holding up to max_keys[i] entries (max_keys == NULL: every
 * heap holds up to max_keys_each).  Returns 0 if k or keytype is
 * unsupported, nheaps is 0 or above 2^20, or a heap would need 2^30 - 1
 * nodes or more. */
uint64_t heap_arena_bytes(uint32_t k, int keytype, uint32_t nheaps, const uint64_t *max_keys,
                          uint64_t max_keys_each);

/* Largest insert one operation may hold (0 for an unsupported k): 4096
 * entries, 2048 for k = 32.  An insert of n > k entries (Sec. 3.2.2, footnote
 * to the INS paragraph: more than k keys are inserted by several INS
 * operations) takes the root once: under that one root hold it runs the root
 * phase of every chunk of k entries in input order (the last chunk may be
 * shorter) exactly as consecutive inserts would, reserving one target per
 * full batch, and the carries of those batches then descend to their targets
 * together, each path node meeting them in chunk order.  The heap is left
 * exactly as by consecutive inserts of the chunks, and the whole insert is
 * linearized at its root ticket.  The insert is rejected whole (sticky
 * GH_ENOMEM) if its batches do not all fit the heap's capacity.  One
 * workgroup then carries every batch through the top levels of the heap, so
 * on a busy heap such operations are slower than k-entry ones (submissions
 * and heap_serve use them only with GH_TUNE_MULTI_INSERT). */
uint32_t heap_insert_max(uint32_t k);

/* Nonzero if the library has a kernel for node capacity k with workgroups
 * of `threads` threads.  Supported k: 32, 64, 128, 256, 512, 1024. */
int heap_supported_shape(uint32_t k, uint32_t threads);

/* Create one heap (Sec. 3.1) of node capacity k and key type keytype
 * (GH_U32_ID or GH_I64_ID) holding up to max_keys entries in the caller's
 * arena d_arena (arena_bytes >= heap_arena_bytes; 256-byte aligned;
 * borrowed, must outlive the handle).  Initializes the arena on `stream`.
 * Errors: GH_EINVAL (also for an unknown keytype), GH_ENOMEM (arena too
 * small), GH_EDEVICE. */
int heap_create(gh_heap_t *out, uint32_t k, uint64_t max_keys, int keytype, void *d_arena,
                uint64_t arena_bytes, void *stream);

/* Create a set of nheaps (1..2^20) independent heaps of node capacity k and
 * key type keytype; heap i holds up to max_keys[i] entries.  Same arena and
 * stream rules as heap_create. */
int heap_create_many(gh_heap_t *out, uint32_t k, int keytype, uint32_t nheaps,
                     const uint64_t *max_keys, void *d_arena,
                     uint64_t arena_bytes, void *stream);

/* Insert n entries from d_keys (device, n entries of the set's width) into heap 0 of the set:
 * ceil(n / k) insert operations of up to k entries each, full chunks first
 * (Sec. 3.2.2 footnote), each run top-down (Sec. 3.3.2) with up to 64 in
 * flight.  (Operations of up to heap_insert_max(k) entries that take the
 * root once are available through heap_submit with GH_TUNE_MULTI_INSERT;
 * they leave the same heap but are slower for bulk inserts.)  n = 0 is a
 * no-op.
 * Errors: GH_EINVAL (null, reserved entry is not checked), GH_ENOMEM (the
 * heap would exceed max_keys; nothing is inserted). */
int heap_insert(gh_heap_t h, const void *d_keys, uint64_t n);

/* Bulk build (Sec. 3.1: a sorted array already satisfies Properties 1-3):
 * heap i of the set, which must be empty, takes the n entries of d_sorted
 * (device, ascending) without any heap operation.  The first floor(n / k) * k
 * entries become the nodes in the order they would have been added (node
 * slot p - 1 holds entries [(p - 1) k, p k); every parent precedes its
 * children in that order), the rest the partial buffer.  n = 0 is a no-op.
 * Errors: GH_EINVAL (null, i out of range; from the device: d_sorted not
 * ascending), GH_ENOMEM (n > max_keys of heap i), GH_ESTATE (from the
 * device: heap i not empty).  Device errors are sticky. */
int heap_build(gh_heap_t h, uint32_t i, const void *d_sorted, uint64_t n);

/* Bytes of device workspace heap_filter needs for heap i of the set (0 for
 * a bad handle or index). */
uint64_t heap_filter_workspace_bytes(gh_heap_t h, uint32_t i);

/* Filter heap i of the set: every entry >= bound is removed (for GH_I64_ID
 * sets every entry whose first word, the biased key, is >= bound; the garbage
 * collection of a branch-and-bound search, Sec. 5.7.2, which drops nodes
 * whose bound can no longer beat the incumbent).  The entries kept are
 * gathered, sorted and laid out again as by heap_build (Sec. 3.1), all on
 * the set's stream; the number kept goes to *d_kept (device, may be NULL).
 * No submission may be in flight on the set (calls on its stream are
 * ordered).  d_work: caller-owned device workspace, 256-byte aligned, at
 * least heap_filter_workspace_bytes(h, i) bytes.  Errors: GH_EINVAL (null
 * handle or workspace, i out of range, workspace too small or misaligned),
 * GH_EDEVICE. */
int heap_filter(gh_heap_t h, uint32_t i, uint64_t bound, void *d_work, uint64_t work_bytes,
                uint64_t *d_kept);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): heap_filter
 * of heap i without a workspace argument.  The workspace is a fixed array of
 * GH_FILTER_NOALLOC_MAX_BYTES in device memory that the library holds on
 * every GPU it runs on until the process ends; its address is looked up when
 * a handle is created on that GPU.  The call allocates nothing: no hipMalloc,
 * no hipFree, no allocating library routine.  Every call on one GPU shares
 * that GPU's array, so calls that can overlap on one GPU (different streams,
 * different handles) race and must be ordered by the caller; calls on one
 * handle are ordered by its stream.  Otherwise as heap_filter: the same
 * kernels, the same result, *d_kept (device, may be NULL) receives the
 * number kept.  Errors: GH_EINVAL (null handle, i out of range), GH_ENOMEM
 * (heap_filter_workspace_bytes(h, i) exceeds GH_FILTER_NOALLOC_MAX_BYTES:
 * heaps of up to about 4 million entries fit), GH_EDEVICE (the array's
 * address could not be found, or a launch failed). */
#define GH_FILTER_NOALLOC_MAX_BYTES (64ull << 20)
int heap_filter_noalloc(gh_heap_t h, uint32_t i, uint64_t bound, uint64_t *d_kept);

/* deleteMin on heap 0 of the set (Sec. 3.2.1, Sec. 3.3.2) of c entries,
 * 1 <= c <= k (the node capacity): writes the min(c, size) smallest entries in
 * ascending order to d_out (device, room for c entries) and that number to
 * *d_count (device).  An empty heap gives *d_count = 0, not an error.  c = k
 * is the paper's deleteMin; for c < k the root's other entries and the
 * partial buffer refill the root, and the last node is taken only when they
 * are fewer than k (the variable-count deleteMin that a heap sharded over
 * several devices needs to remove a globally selected share).
 * Errors: GH_EINVAL (null pointer, c = 0 or c > k). */
int heap_delete_min(gh_heap_t h, void *d_out, uint32_t c, uint32_t *d_count);

/* Run nops operations (d_ops, device) on the set's heaps in one persistent
 * launch with many operations in flight (Sec. 3.3): each workgroup claims the
 * next operation in list order, waits for its arrival time, takes the heap's
 * root in `seq` order, and runs the operation top-down under node locks.
 * Inserts read d_in, deleteMins write d_out and d_counts[i] (device, one
 * uint32 per operation; inserts get 0); d_log (device, nops records, may be
 * NULL) receives one gh_logrec per operation.  Capacity overruns are
 * detected on the device (sticky GH_ENOMEM).  nops < 2^24. */
int heap_submit(gh_heap_t h, const gh_op *d_ops, uint32_t nops,
                const void *d_in, void *d_out, uint32_t *d_counts,
                gh_logrec *d_log, const gh_tuning *tuning);

/* Like heap_submit, but records the launch into a HIP graph once and returns
 * it as *graph_out (a hipGraphExec_t passed as void*); heap_graph_launch
 * replays it on the set's stream with the same arguments, and
 * heap_graph_destroy frees it. */
int heap_submit_graph(gh_heap_t h, const gh_op *d_ops, uint32_t nops,
                      const void *d_in, void *d_out, uint32_t *d_counts,
                      gh_logrec *d_log, const gh_tuning *tuning, void **graph_out);
int heap_graph_launch(gh_heap_t h, void *graph);
int heap_graph_destroy(void *graph);

/* Bytes of device workspace heap_serve needs for nreq requests that expand
 * into at most max_ops operations on a set of nheaps heaps; 0 if nheaps is
 * 0 or above 2^20, or max_ops is 0 or above 2^24 - 1 (heap_serve's limits). */
uint64_t heap_serve_workspace_bytes(uint32_t nheaps, uint32_t nreq, uint64_t max_ops);

/* Serve a request stream with a device-resident loop (one persistent
 * launch).  d_reqs (device, nreq gh_op records, non-decreasing arrival_ns;
 * `seq` is ignored) are requests: an insert of any n >= 0 entries from
 * d_in + off, or a deleteMin of n entries (1..k, 0 meaning k; a larger n
 * is rejected with GH_EINVAL) writing up to that many to d_out + off.
 * Workgroup 0 admits requests in arrival order once their arrival time has
 * passed: a deleteMin always, an insert when the heap's size after all
 * admitted requests plus n stays within the heap's max_keys; otherwise the
 * insert waits (per heap, first in first out) until admitted deleteMins make
 * room.  Each heap's admitted requests take the root in admission order, so
 * a heap's results do not depend on the other heaps in the stream (while
 * max_ops has room for every admitted operation).  Admitted requests become
 * operations (a deleteMin, or an insert cut into operations of k entries,
 * each its own root turn) that the other workgroups (the slots,
 * tuning->workgroups of them) run as in heap_submit.  With
 * GH_TUNE_MULTI_INSERT in tuning->flags an insert is cut into operations of
 * up to heap_insert_max(k) entries instead, each taking the root once (the
 * results are the same; the carries of one operation then descend in one
 * slot, one after another, which lowers the throughput of a busy heap).
 * d_recs (device, nreq records) receives one gh_reqrec per request.
 * d_work is a caller-owned device workspace of heap_serve_workspace_bytes.
 * The scheduler keeps 32 bytes per heap in LDS: nheaps * 32 + threads * 8 +
 * k * 5 * (entry bytes) + 1024 must not exceed 64 KiB (1024 heaps at
 * k = 256 with 8-byte entries; 256 heaps at k = 1024).
 * Errors: GH_EINVAL (bad sizes, max_ops too small is reported as a sticky
 * GH_ENOMEM and the requests that did not fit are rejected). */
int heap_serve(gh_heap_t h, const gh_op *d_reqs, uint32_t nreq, const void *d_in,
               void *d_out, gh_reqrec *d_recs, void *d_work, uint64_t work_bytes,
               uint64_t max_ops, const gh_tuning *tuning);

/* Result of one knapsack instance solved by heap_knapsack (64 bytes).
 *   best        optimal value found
 *   explored    nodes taken from the heap and expanded (bound above best)
 *   created     nodes pushed into the heap
 *   popped      nodes taken from the heap by the search (the search stops
 *               before popping those whose bound cannot beat best)
 *   gc_dropped  heap entries removed by garbage collections
 *   alg_bytes   algorithmic bytes of the instance's heap operations (as
 *               gh_reqrec.bytes; a collection adds 2e per entry kept)
 *   ops         heap operations the instance ran (inserts, deleteMins and
 *               the operations of its collections)
 *   flags       bit 0: finished; bit 5: refused (more than 255 items, a
 *               capacity of 2^28 or more, or values summing beyond what the
 *               entry encodes: 2^18 for GH_U32_ID sets, 2^28 for GH_I64_ID);
 *               bit 6: the node pool overflowed (best is then only a lower
 *               bound)
 *   gc_runs     garbage collections of the instance's heap */
typedef struct gh_knapres {
    uint64_t best;
    uint64_t explored;
    uint64_t created;
    uint64_t popped;
    uint64_t gc_dropped;
    uint64_t alg_bytes;
    uint32_t ops;
    uint32_t flags;
    uint32_t gc_runs;
    uint32_t reserved;
} gh_knapres;

/* Solve ninst 0/1 knapsack instances by best-first branch and bound, one
 * heap of the set per instance, all in one persistent launch (the
 * application of Sec. 5.7.2).  Instance i has d_n[i] <= 255 items starting
 * at d_item_off[i] in d_w / d_v (uint32, sorted by value/weight
 * descending), capacity d_cap[i] < 2^28.  A heap entry orders the search
 * nodes by their fractional upper bound in fixed point (scale 2^16), largest
 * first: in a GH_I64_ID set the key is the negated bound as a signed 64-bit
 * integer and the id the node's pool index; in a GH_U32_ID set the entry
 * packs (2^35 - 1 - bound) above a 29-bit pool index.  So deleteMin returns
 * the k most promising nodes; a node is expanded only if its bound exceeds
 * the best value found, children are pushed only if their bound does, and an
 * instance stops (its heap emptied without reading the rest) once the best
 * bound left cannot beat the best value found.  Garbage collection (Sec.
 * 5.7.2): with gc_min > 0, when an instance's heap holds gc_min entries or
 * more and the best value has improved since its last collection, every
 * entry whose bound cannot beat the best value leaves the heap (the kept
 * entries are laid out as by heap_build); it runs only when nodes that are
 * entirely dead hold at least a quarter of the heap and the heap's free
 * node slots can stage the kept entries.  gc_min = 0 never collects.
 * d_pool (device, ninst * pool_per_inst uint64) holds the nodes; d_scratch
 * (device, ninst * 3 * k entries of the set's width) holds per-instance
 * batches; d_res (device, ninst gh_knapres).  Heap i must hold
 * pool_per_inst entries (pool_per_inst < 2^29 for GH_U32_ID sets, < 2^32
 * for GH_I64_ID).  An instance beyond the limits above or the entry's value
 * range is refused on the device (flags bit 5, sticky GH_EINVAL).
 * Instances are claimed by the workgroups in order; a submission may not
 * overlap another submission on the same set.  Errors: GH_EINVAL,
 * GH_ENOMEM (a heap smaller than pool_per_inst). */
int heap_knapsack(gh_heap_t h, uint32_t ninst, const uint32_t *d_item_off,
                  const uint32_t *d_n, const uint64_t *d_cap, const uint32_t *d_w,
                  const uint32_t *d_v, uint64_t *d_pool, uint64_t pool_per_inst,
                  void *d_scratch, gh_knapres *d_res, uint32_t gc_min,
                  const gh_tuning *tuning);

/* Counters of a heap_sssp run (72 bytes, device memory).
 *   popped      entries taken from the heap
 *   stale       popped entries whose distance had already improved (skipped)
 *   pushed      entries inserted (each a strict improvement of a distance)
 *   heap_ops    heap operations (inserts + deleteMins)
 *   heap_ticks, relax_ticks  device wall-clock ticks summed over workgroups
 *               spent in heap operations and in edge relaxation
 *   rounds      deleteMins that returned entries
 *   traced      heap operations the trace asked to record (0 without a
 *               trace; more than trace->op_cap means the trace is cut)
 *   alg_bytes   algorithmic bytes of the heap operations (as
 *               gh_reqrec.bytes) */
typedef struct gh_ssspstats {
    uint64_t popped;
    uint64_t stale;
    uint64_t pushed;
    uint64_t heap_ops;
    uint64_t heap_ticks;
    uint64_t relax_ticks;
    uint64_t rounds;
    uint64_t traced;
    uint64_t alg_bytes;
} gh_ssspstats;

/* One heap operation of a traced SSSP run (32 bytes): its root ticket, its
 * kind (GH_OP_INSERT / GH_OP_DELETE_MIN), the entry count (inserted, or
 * returned), and where its entries start in the trace's key buffer
 * (inserts: the batch as given, unsorted; deleteMins: the output).
 * `reserved` = m << 32 | s << 16 | flags << 8 | levels: the node count and
 * partial-buffer size seen at the root, and the gh_logrec flags and levels. */
typedef struct gh_ssspop {
    uint64_t ticket;
    uint64_t off;
    uint32_t count;
    uint32_t kind;
    uint64_t reserved;
} gh_ssspop;

/* Optional trace of an SSSP run (host struct naming device buffers): room
 * for op_cap records and key_cap entries.  Records come in completion
 * order; sorted by ticket they replay the run on a sequential heap
 * (Theorem 1).  An operation that does not fit is not recorded (the stats'
 * `traced` count tells); the source's insert (the run's first ticket) is
 * not recorded. */
typedef struct gh_sssptrace {
    gh_ssspop *d_ops;
    uint64_t op_cap;
    uint64_t *d_keys;
    uint64_t key_cap;
} gh_sssptrace;

/* Single-source shortest paths (the application of Sec. 5.7.1) with heap 0
 * of a GH_U32_ID set (GH_EINVAL for other key types) as a shared priority
 * queue: entries are dist << 32 | vertex;
 * every workgroup repeatedly takes the k nearest entries, skips those whose
 * vertex has since been reached by a shorter path, relaxes the out-edges of
 * the rest with an atomic minimum on the distance, and inserts an entry for
 * every strict improvement.  Many workgroups use the heap at once.  The run
 * ends when the heap is empty and no workgroup holds entries.  Graph in CSR
 * (device): d_rowptr[V + 1], d_col / d_w[E] (uint32 weights); distances
 * must stay below 2^32 - 1; d_dist[V] receives the distances (UINT32_MAX =
 * unreachable).  An edge whose target is not below V is skipped and the run
 * reports GH_EINVAL; rowptr must be non-decreasing with rowptr[V] = E (not
 * checked on the device).  d_push (device) holds workgroups * (push_per_wg + k)
 * entries (workgroups = tuning->workgroups, 256 when 0 or tuning is NULL);
 * push_per_wg >= k * (largest out-degree) guarantees room for one round of
 * improvements, else the run stops with GH_ENOMEM.  Heap 0 must be empty;
 * the run stops with GH_ENOMEM if the live entries outgrow its capacity
 * (E + 1 entries is ample: live entries are far fewer than pushes).
 * d_stats: one gh_ssspstats (device).  trace (host struct, may be NULL):
 * record every heap operation (slower; for verification).  Asynchronous on
 * the set's stream; errors surface at heap_sync.  The heap is empty again
 * afterwards. */
int heap_sssp(gh_heap_t h, uint32_t V, const uint32_t *d_rowptr, const uint32_t *d_col,
              const uint32_t *d_w, uint32_t src, uint32_t *d_dist, uint64_t *d_push,
              uint64_t push_per_wg, gh_ssspstats *d_stats, const gh_tuning *tuning,
              const gh_sssptrace *trace);

/* Wait for the set's stream; return the sticky device error (GH_OK if none). */
int heap_sync(gh_heap_t h);

/* Synchronous: wait for the stream and write heap i's entry count to
 * *out_host (host memory). */
int heap_size(gh_heap_t h, uint32_t i, uint64_t *out_host);

/* Synchronous: copy heap i's state to host memory for inspection:
 * meta_host[0..3] = {nodes in use m, partial-buffer size s, tickets served,
 * node capacity}; nodes_host (may be NULL) receives max_nodes * k entries
 * of the set's width,
 * slot p-1 holding the node added p-th (bit-reversal order, Sec. 4.3);
 * pb_host (may be NULL) receives s entries (s < k: room for k - 1 entries
 * always suffices). */
int heap_read_state(gh_heap_t h, uint32_t i, uint64_t *meta_host,
                    void *nodes_host, void *pb_host);

/* Synchronous: wait for the stream, release the handle, and return the
 * sticky device error.  The arena may be freed afterwards. */
int heap_destroy(gh_heap_t h);

/* Static description of an error code. */
const char *heap_strerror(int code);

/* Device wall-clock frequency in Hz (for gh_logrec timestamps). */
uint64_t heap_clock_hz(void);

#ifdef __cplusplus
}
#endif

#endif /* GHEAP_H */
