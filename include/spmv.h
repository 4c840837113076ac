/*
 * spmv.h -- C ABI of the MI355X (gfx950) row-partitioned SpMV library.
 *
 * The library computes one rank's share of the distributed sparse
 * matrix-vector product y = A x of Sec. III-A of "Machine Learning for
 * CUDA+MPI Design Rules" (Pearson, Javeed, Devine): the rows, x entries and
 * y entries of A are divided into contiguous blocks over P ranks; rank r
 * computes y_r = A_L x_L + A_R x_R, where A_L holds the columns of the x
 * entries it owns and A_R the columns owned by other ranks.  One exec runs
 * the operations of the paper's SpMV program DAG (Fig. 3c):
 *
 *   Pack      gather the owned x entries other ranks need into one send
 *             buffer per destination (GPU kernel)
 *   y_L       local CSR product A_L x_L (GPU kernel)
 *   PostSend  start sending the packed buffers (here: asynchronous copy of
 *             the send buffer into a pinned host outbox)
 *   PostRecv  start receiving the halo x_R (here: asynchronous copy of a
 *             pinned host inbox, filled by the caller, into device memory)
 *   WaitSend / WaitRecv   block the host until the copy finished
 *   Unpack    place received values in halo order (GPU kernel)
 *   y_R       remote CSR product A_R x_R, added into y (GPU kernel)
 *   start / end           artificial entry and exit; end waits for all work
 *
 * The order of these operations and the stream each GPU operation runs on
 * are an explicit plan input (a traversal of the DAG, Sec. III-B), and the
 * synchronisation operations of Table III are explicit tokens of that order.
 * On one GPU the other ranks are emulated: the caller fills the inbox with
 * the halo values and reads the packed values from the outbox.
 *
 * Conventions
 *   - All functions return an int status: SPMV_OK (0) or a negative
 *     SPMV_E* code; spmv_last_error() then gives a message (thread-local,
 *     valid until the next call on the same thread).  No C++ exception
 *     crosses this boundary.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory on the current device.  Streams are hipStream_t passed
 *     as void* (NULL = the null stream).
 *   - Matrices are CSR with int32 row_ptr/col_idx and FP64 values; column
 *     indices strictly ascending inside each row.
 *   - A plan is not safe for concurrent use from several host threads.
 */
#ifndef SPMV_H
#define SPMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define SPMV_OK       0
#define SPMV_EINVAL  -1   /* NULL pointer, size or index out of range        */
#define SPMV_ECSR    -2   /* malformed CSR: row_ptr not monotone, column out
                             of range, columns unsorted or duplicated         */
#define SPMV_EPLAN   -3   /* invalid operation order / stream map            */
#define SPMV_ENOMEM  -4   /* host or device allocation failed                */
#define SPMV_EHIP    -5   /* a HIP runtime call failed (message names it)    */
#define SPMV_EBUDGET -6   /* serving: request does not fit the memory budget */
#define SPMV_ESTATE  -7   /* call not valid in the object's current state    */

/* ------------------------------------------------------------ operations
 * DAG vertices of the SpMV program (Sec. III-A).  Table II types:
 * CPU = start, PostSend, PostRecv, WaitSend, WaitRecv, end;
 * GPU = Pack, y_L, Unpack, y_R (bound to a stream by the stream map).     */
#define SPMV_OP_START      0
#define SPMV_OP_PACK       1
#define SPMV_OP_YL         2
#define SPMV_OP_POST_SEND  3
#define SPMV_OP_POST_RECV  4
#define SPMV_OP_WAIT_SEND  5
#define SPMV_OP_WAIT_RECV  6
#define SPMV_OP_UNPACK     7
#define SPMV_OP_YR         8
#define SPMV_OP_END        9
#define SPMV_N_VERTICES   10

/* Synchronisation operations of Table III, inserted for a DAG edge u -> v:
 *   GPU u -> CPU v:               CER-after-u, then CES-b4-v
 *                                 (event record on u's stream; the host
 *                                 blocks on that event before v)
 *   GPU u -> GPU v, other stream: CER-after-u, then CSWE-b4-v
 *                                 (v's stream waits on the event)
 *   CPU u -> anything, GPU u -> GPU v on u's stream: nothing.
 * A record captures all work issued to u's stream before the record token,
 * not only u.  Edges into end need no tokens: end waits for everything.   */
#define SPMV_SYNC_CER    0x10
#define SPMV_SYNC_CES    0x20
#define SPMV_SYNC_CSWE   0x30
#define SPMV_CER_AFTER(u)  (SPMV_SYNC_CER  | (u))
#define SPMV_CES_B4(v)     (SPMV_SYNC_CES  | (v))
#define SPMV_CSWE_B4(v)    (SPMV_SYNC_CSWE | (v))

/* Fine-grained program (Sec. III-A): one Pack, PostSend and WaitSend per
 * destination rank q and one PostRecv and WaitRecv per source rank q, token
 * SPMV_PEER(op, q); start, y_L, y_R and end are shared, Unpack is implied
 * before y_R, and the synchronisation macros above wrap peer tokens too
 * (SPMV_CER_AFTER(SPMV_PEER(SPMV_OP_PACK, q)), ...).                      */
#define SPMV_PEER(op, q)   ((op) | (((q) + 1) << 8))

#define SPMV_MAX_OPS     24   /* longest valid coarse operation order       */
#define SPMV_MAX_STREAMS  8

/* ------------------------------------------------------------ types */

/* Global matrix, host memory, borrowed for the duration of the call. */
typedef struct {
    int32_t        n_rows;
    int32_t        n_cols;    /* must equal n_rows (square, same partition) */
    int64_t        nnz;
    const int32_t *row_ptr;   /* [n_rows + 1], row_ptr[0] = 0               */
    const int32_t *col_idx;   /* [nnz], ascending inside each row           */
    const double  *val;       /* [nnz]                                      */
} spmv_csr_t;

/* Kernel variant knobs (not part of the paper's plan; chosen by the tuner).
 * Zero-initialised = automatic choice for every field.
 *
 * Two CSR kernel families compute y_L and y_R:
 *   vector CSR  each row is reduced by a group of `lanes` lanes; each lane
 *               group handles `rows` rows with all their loads in flight
 *   stream CSR  rows are cut into tiles whose entries fit one window of
 *               256 * `chunk` entries; the block streams the window with
 *               `width`-entry loads, stages the products in LDS and `lanes`
 *               lanes per row sum them                                       */
#define SPMV_KERNEL_VECTOR 1
#define SPMV_KERNEL_STREAM 2

typedef struct {
    int32_t kernel_local;  /* 0 = auto, 1 = vector CSR, 2 = stream CSR      */
    int32_t kernel_remote; /* same for y_R                                   */
    int32_t lanes_local;   /* lanes per row: 0 = auto, 1..64 pow2 (stream:
                              1..16)                                         */
    int32_t lanes_remote;
    int32_t rows_local;    /* vector: rows per lane group, 0 = auto, 1/2/4/8 */
    int32_t rows_remote;   /* same for y_R; in column slabs (form 5) rows per
                              thread: 0/1 = tiles of 256 / lanes_remote rows,
                              2/4/8 = wide tiles of up to that many times 256
                              rows, one thread per row (lanes_remote 0 or 1) */
    int32_t chunk_local;   /* stream: entries per thread per window, 0 = auto,
                              4, 8 or 16                                      */
    int32_t chunk_remote;
    int32_t width;         /* stream: entries per load, 0 = auto, 2 or 4     */
    int32_t xcd_remap;     /* 0 = auto, 1 = contiguous row tiles per XCD,
                              2 = plain round-robin block order             */
    int32_t fuse_unpack;   /* 0 = auto: y_R reads the receive buffer in
                              place whenever the unpack permutation is the
                              identity (always here: the receive layout
                              equals the halo order), so no Unpack kernel
                              runs; 1 = fused (SPMV_EINVAL if the permutation
                              is not the identity); 2 = the explicit Unpack
                              kernel                                         */
    int32_t flags;         /* SPMV_F_* below                               */
    int32_t form;          /* stream: 1 = packed tiles (rows cut to fill
                              each window), 2 = sliced ELL (a wave per 64
                              rows, entries stored column-major per slice,
                              each row an fma chain; taken only when padding
                              stays within 15%, else packed tiles; chunk =
                              entries per batch of loads: 4, 8, 16),
                              3 = sliced ELL whose y_L columns are stored as
                              16-bit offsets from the row, 8 per lane per
                              16-byte load, and values in pairs, 2 per lane
                              per 16-byte load (taken when every slice has one
                              width and every |col - row| <= 32767, else
                              form 2; y_R takes form 2; chunk 8 or 16),
                              4 = packed tiles whose y_L columns are stored
                              as 16-bit offsets from the first row of their
                              tile (taken when every offset fits, else form
                              1; y_R takes form 1), 0 = auto: sliced when
                              every slice of 64 rows has the same width of
                              at most 8, else packed, y_L with 16-bit
                              offsets (forms 3, 4) when they fit.
                              5 = y_R in column slabs: the halo cut into 8
                              equal column ranges, one per XCD, so the x
                              values a slab gathers stay in one XCD's L2;
                              each slab in packed tiles writes a partial sum
                              per row, and a second kernel adds a row's 8
                              partial sums in slab order (lanes_remote at
                              most 4; y_L takes the automatic form; without
                              remote rows y_R stays in form 1).  The
                              automatic form (0) takes column slabs for y_R
                              when the halo (8 bytes per entry) exceeds one
                              XCD's 4 MiB L2 and y_R uses the stream kernel.
                              Every form but 5 gives the same bits for y;
                              form 5 gives bits of its own, the same under
                              every plan.  Plans in forms 1 and 4 can join
                              a batch.                                     */
} spmv_tune_t;

#define SPMV_F_HOST_ONLY  1  /* build metadata only: no device resources;
                                inspection works, spmv_exec returns
                                SPMV_ESTATE                                  */
#define SPMV_F_PROFILE    2  /* time every GPU op and copy with HIP events   */
#define SPMV_F_NO_BUFFER  4  /* CSR kernels address memory with 64-bit
                                pointers instead of buffer resources (the
                                latter is used when every array < 4 GiB)     */
#define SPMV_F_RESIDENT_SEQUENTIAL 8  /* spmv_exec_resident launches each op
                                on its own even where it could group them
                                (same bits)                                  */

typedef struct spmv_plan  spmv_plan_t;   /* opaque */

typedef struct {
    int64_t n_global;      /* rows of A                                     */
    int64_t lo;            /* first owned global row                        */
    int64_t n_loc;         /* owned rows                                    */
    int64_t nnz_local;     /* entries of A_L                                */
    int64_t nnz_remote;    /* entries of A_R                                */
    int64_t n_halo;        /* |x_R|: distinct remote columns                */
    int64_t n_send;        /* total entries packed for other ranks          */
    int64_t n_remote_rows; /* owned rows with at least one remote entry     */
    int64_t device_bytes;  /* device memory owned by the plan               */
    int32_t nranks, rank;
    int32_t n_streams;     /* plan streams (stream 0 = the caller's; copy
                              streams not counted)                          */
    int32_t n_ops;         /* tokens in the canonical operation order        */
    int32_t kernel_local, kernel_remote;   /* 1 = vector CSR, 2 = stream CSR */
    int32_t lanes_local, lanes_remote, rows_local, rows_remote;
    int32_t chunk_local, chunk_remote, width;
    int32_t xcd_remap, fuse_unpack;
    int32_t fused_combine; /* 1: y_R adds into y itself; 0: a combine step
                              at end adds the remote partial sums            */
    int32_t n_tiles_local, n_tiles_remote;  /* packed stream tiles (0: none;
                              form 5: the tiles of all 8 slabs)            */
    int32_t form_local;    /* y_L stream form: 1 packed tiles, 2 sliced ELL,
                              3 sliced ELL with 16-bit column offsets,
                              4 packed tiles with 16-bit column offsets,
                              5 column slabs (y_R), 0 vector CSR            */
    int32_t form_remote;   /* same for y_R                                   */
    int32_t n_slices_local, n_slices_remote;  /* sliced-ELL slices (0: none) */
    int32_t fine;          /* 1 while a fine-grained order is in force       */
    int32_t device;        /* HIP device of the plan's memory (-1 host-only) */
    int32_t resident_grouped; /* launches of spmv_exec_resident: 1 = the two
                              grouped launches, 3 = one launch (y_L's, with
                              Pack and the remote sums), 2 = Pack as extra
                              blocks of y_L's launch, then y_R, 0 = one per
                              op (see spmv_exec_resident)                   */
} spmv_info_t;

/* Integer metadata selectors for spmv_plan_get_i32. */
#define SPMV_I32_HALO_COLS    0  /* [n_halo] global columns of x_R, ascending */
#define SPMV_I32_RECV_OFF     1  /* [nranks+1] halo entries owned by rank q:
                                    [recv_off[q], recv_off[q+1])             */
#define SPMV_I32_SEND_IDX     2  /* [n_send] local x indices packed, grouped
                                    by destination ascending, ascending      */
#define SPMV_I32_SEND_OFF     3  /* [nranks+1]                                */
#define SPMV_I32_AL_PTR       4  /* [n_loc+1] A_L row pointer                 */
#define SPMV_I32_AL_COLS      5  /* [nnz_local] local column indices          */
#define SPMV_I32_AR_ROWS      6  /* [n_remote_rows] local row ids, ascending  */
#define SPMV_I32_AR_PTR       7  /* [n_remote_rows+1]                         */
#define SPMV_I32_AR_COLS      8  /* [nnz_remote] index into the halo          */
#define SPMV_I32_UNPACK_PERM  9  /* [n_halo] x_halo[p] = recv[perm[p]]        */
#define SPMV_I32_OP_ORDER    10  /* [n_ops] canonical operation order          */
#define SPMV_I32_STREAM_MAP  11  /* [SPMV_N_VERTICES] canonical streams, -1
                                    for CPU vertices                          */
#define SPMV_I32_TILE_ROW_L  12  /* [n_tiles_local+1] stream-CSR tile rows of
                                    A_L: tile t = rows [row[t], row[t+1])     */
#define SPMV_I32_TILE_K_L    13  /* [n_tiles_local+1] first entry of each tile */
#define SPMV_I32_TILE_ROW_R  14  /* same for A_R (compressed rows); in column
                                    slabs (form 5) the 8 slabs' arrays one
                                    after another, each closed by its own
                                    last entry: n_tiles_remote + 8 in all,
                                    entries counted within the slab         */
#define SPMV_I32_TILE_K_R    15
#define SPMV_I32_OP_STREAM   16  /* [n_ops] canonical stream of each position of
                                    the order in force, -1 for tokens that
                                    run on no plan stream                     */

/* FP64 selectors for spmv_plan_get_f64 (device contents are copied back). */
#define SPMV_F64_AL_VAL       0  /* [nnz_local]                               */
#define SPMV_F64_AR_VAL       1  /* [nnz_remote]                              */
#define SPMV_F64_SENDBUF      2  /* [n_send] device send buffer after Pack    */
#define SPMV_F64_RECVBUF      3  /* [n_halo] device receive buffer            */
#define SPMV_F64_X_HALO       4  /* [n_halo] x_R after Unpack (the receive
                                    buffer itself when Unpack is fused)       */
#define SPMV_F64_OP_MS        5  /* [SPMV_N_VERTICES + 1] summed milliseconds
                                    per op since the last reset (SPMV_F_PROFILE;
                                    index SPMV_N_VERTICES = combine step)      */
#define SPMV_F64_OP_COUNT     6  /* [SPMV_N_VERTICES + 1] timed launches       */
#define SPMV_F64_HOST_US      7  /* [n_ops] summed microseconds from an exec's
                                    entry to the return of each token's host
                                    call, in order (host timeline, profile
                                    mode 2); cleared when the order changes  */
#define SPMV_F64_HOST_COUNT   8  /* [1] execs summed in SPMV_F64_HOST_US      */

/* ------------------------------------------------------------ plans */

/*
 * Build rank `rank`'s share of `csr` partitioned over `nranks` contiguous row
 * blocks (rank q owns rows [q*floor(n/P) + min(q, n mod P), ...)), split it
 * into A_L / A_R (Sec. III-A), derive the halo set and the send lists,
 * validate the operation order, and allocate and upload everything the exec
 * needs: device CSRs, send/receive buffers, pinned inbox/outbox and the
 * events.  Plan streams other than stream 0 (which is the caller's stream
 * at exec time) and the copy streams come from a per-device pool shared by
 * all plans.
 *
 *   csr        host, borrowed; validated (SPMV_ECSR on any defect)
 *   nranks     >= 1; rank in [0, nranks)
 *   op_order   host [n_ops] operation tokens (SPMV_OP_*, SPMV_CER_AFTER(u),
 *              SPMV_CES_B4(v), SPMV_CSWE_B4(v)), or NULL for the default plan.
 *              Must be a topological order of the DAG that starts with
 *              START, ends with END and contains exactly the Table III
 *              tokens its stream binding requires (SPMV_EPLAN otherwise).
 *              UNPACK may be omitted: it is then run on y_R's stream
 *              immediately before y_R.  With nranks == 1 the DAG is
 *              START -> y_L -> END.
 *   stream_map host [SPMV_N_VERTICES] stream of each GPU vertex (indexed by
 *              SPMV_OP_*; entries of CPU vertices are ignored), values in
 *              [0, n_streams); NULL = all on stream 0.  Streams are
 *              relabelled by first use along the order (plans equal up to a
 *              stream bijection are the same plan).
 *   n_streams  1..SPMV_MAX_STREAMS plan streams
 *   tune       kernel knobs, NULL = automatic
 *   out        receives the plan; the caller owns it (spmv_plan_destroy)
 *
 * The caller may free every input on return.
 */
int spmv_plan_create(const spmv_csr_t *csr, int32_t nranks, int32_t rank,
                     const int32_t *op_order, int32_t n_ops,
                     const int32_t *stream_map, int32_t n_streams,
                     spmv_plan_t **out);
int spmv_plan_create_ex(const spmv_csr_t *csr, int32_t nranks, int32_t rank,
                        const int32_t *op_order, int32_t n_ops,
                        const int32_t *stream_map, int32_t n_streams,
                        const spmv_tune_t *tune, spmv_plan_t **out);

/*
 * Same as spmv_plan_create_ex, from what one rank of a distributed code
 * holds instead of the global matrix: its own rows and its send lists.
 *   local      host CSR of the rank's n_loc rows (n_rows = n_loc of the
 *              contiguous partition of n_global rows over nranks) with
 *              GLOBAL column indices (n_cols = n_global), ascending per row
 *   send_idx   host [send_off[nranks]] local indices of owned x entries that
 *              each other rank needs, ascending per destination,
 *              destinations ascending (the rank itself gets none)
 *   send_off   host [nranks + 1]
 * The halo is derived from the local rows as in the global form.
 */
int spmv_plan_create_local(const spmv_csr_t *local, int64_t n_global, int32_t nranks,
                           int32_t rank, const int32_t *send_idx, const int32_t *send_off,
                           const int32_t *op_order, int32_t n_ops, const int32_t *stream_map,
                           int32_t n_streams, const spmv_tune_t *tune, spmv_plan_t **out);

/* Release everything the plan owns.  NULL-safe. */
int spmv_plan_destroy(spmv_plan_t *plan);

/*
 * One SpMV of the rank share: y_local = (A x)[lo, lo + n_loc).
 *
 *   x_local  device [n_loc] owned x entries (read only)
 *   y_local  device [n_loc] result; must not alias x_local
 *   stream   ordering anchor and plan stream 0: the plan's stream-0 steps
 *            run on `stream` itself, after work already issued to it; the
 *            other plan streams wait for that work at start, and `stream`
 *            waits for them at end (a one-stream plan records no start or
 *            end events)
 *
 * The halo values are read from the plan's pinned inbox, which the caller
 * fills beforehand (spmv_plan_inbox) with x at the halo columns, in halo
 * order (the values the other ranks would send).  On return the outbox
 * (spmv_plan_outbox) holds the packed send buffer.  The call runs the plan's
 * operation order token by token and returns after end, i.e. with all work
 * finished (host-synchronous, like the paper's end vertex).  Every plan
 * gives bit-identical y: y[i] = fl(s_L[i] + s_R[i]) where the two partial
 * sums do not depend on the plan.
 */
int spmv_exec(spmv_plan_t *plan, const double *x_local, double *y_local, void *stream);

/*
 * The share's device work alone, for a halo that is already in device
 * memory (the receive buffer, spmv_plan_device_buffers: filled by an
 * earlier spmv_exec, or written there by the caller, e.g. from a
 * device-to-device exchange): Pack into the device send buffer, y_L,
 * Unpack, y_R adding into y, launched on `stream` and returning at once
 * (asynchronous; no copies, no host waits, no other stream).  The launches
 * (spmv_info_t.resident_grouped):
 *   1  y_R in column slabs, y_L in packed tiles of the same window and
 *      width, Unpack fused: two grouped launches, Pack, y_L and the slab
 *      tiles (none reads what another writes) as the work items of one,
 *      then the slab sums adding into y;
 *   3  y_L in packed tiles or the 16-bit sliced form, Unpack fused, y_R
 *      sliced or in packed tiles with one summing lane, and either both in
 *      packed tiles with at most one window (and at most 1,024) of remote
 *      entries in the rows of each y_L tile, or no remote row longer than 4
 *      entries: the whole step in y_L's launch, Pack as extra blocks and
 *      each row's remote sum (computed as y_R's kernel computes it) added
 *      where the row's local sum is stored;
 *   2  otherwise, with y_L in packed tiles or the 16-bit sliced form: Pack
 *      as extra blocks of y_L's launch, then Unpack (unless fused) and y_R;
 *   0  otherwise, and always with SPMV_F_RESIDENT_SEQUENTIAL: one launch
 *      per op in the DAG's order.
 * y has the bits spmv_exec gives for the same halo in every case.  x_local, y_local as in spmv_exec.  The Sec. III-A
 * product with its exchange taken out: what one rank's GPU computes once
 * its halo has arrived.
 */
int spmv_exec_resident(spmv_plan_t *plan, const double *x_local, double *y_local, void *stream);

/*
 * One of the two grouped launches of spmv_exec_resident, for timing them
 * apart: part 0 = Pack, y_L and the column-slab tiles (y_L stores its row
 * sums into y, the slab tiles their partial sums into the plan's device
 * buffer), part 1 = the slab sums adding into y (after part 0 of the same
 * plan).  Asynchronous on `stream`.  SPMV_ESTATE when the plan's resident
 * step is not grouped (spmv_info_t.resident_grouped = 0), SPMV_EINVAL for
 * another part or NULL / aliasing vectors.
 */
int spmv_exec_resident_part(spmv_plan_t *plan, int32_t part, const double *x_local,
                            double *y_local, void *stream);

/*
 * Device addresses of the plan's send buffer (n_send doubles, written by
 * Pack) and receive buffer (n_halo doubles, read by Unpack / y_R, in halo
 * order), for callers that move the halo themselves.  Owned by the plan.
 */
int spmv_plan_device_buffers(const spmv_plan_t *plan, double **send_dev, int64_t *n_send,
                             double **recv_dev, int64_t *n_halo);

/*
 * Launch one GPU operation of the plan on `stream`, asynchronously: no
 * synchronisation token, no copy, no host wait.  For callers that compose
 * their own schedule (or capture one in a graph) and for kernel timing.
 *   SPMV_OP_PACK    send buffer <- x_local[send_idx]
 *   SPMV_OP_YL      y_local = A_L x_local
 *   SPMV_OP_UNPACK  x_halo <- receive buffer (permuted)
 *   SPMV_OP_YR      y_local[rows of A_R] += A_R x_halo; the caller orders it
 *                   after y_L on the same stream (or after a join)
 * x_local / y_local as in spmv_exec (only the ones the op touches are read).
 */
int spmv_op_launch(spmv_plan_t *plan, int32_t op, const double *x_local, double *y_local,
                   void *stream);

/*
 * Replace the plan's operation order and stream map (same rules and errors as
 * spmv_plan_create), keeping the uploaded share.  The plan owns
 * max(n_streams given at creation, streams the order uses) plan streams; an
 * order that needs more returns SPMV_EPLAN.  For sweeping the design space
 * over one matrix.  On error the previous order stays in force.
 */
int spmv_plan_reorder(spmv_plan_t *plan, const int32_t *op_order, int32_t n_ops,
                      const int32_t *stream_map, int32_t n_streams);

/*
 * The paper's benchmark protocol (Sec. III-C3): a measurement repeats the
 * program (a sample) until t_measure seconds have elapsed on the host clock
 * and records elapsed / samples; n_measure measurements are written to host
 * times[0..n_measure) in seconds.  Sample i runs spmv_exec(plans[i % n_plans],
 * x[i % n_plans], y[i % n_plans], stream): with n_plans = 1 this is the
 * paper's protocol on one plan; with several replicas of one share (same
 * order and streams) the samples rotate over independent device copies,
 * which keeps the matrix out of the last-level cache between samples.  The
 * call first waits for the whole device to go idle (hipDeviceSynchronize).
 */
int spmv_plan_time(spmv_plan_t *const *plans, int32_t n_plans, const double *const *x,
                   double *const *y, void *stream, double t_measure, int32_t n_measure,
                   double *times);

int spmv_plan_info(const spmv_plan_t *plan, spmv_info_t *info);

/* Copy integer metadata `which` (SPMV_I32_*) into host out[0..n); n must be
 * at least the selected array's length (SPMV_EINVAL otherwise). */
int spmv_plan_get_i32(const spmv_plan_t *plan, int32_t which, int32_t *out, int64_t n);
/* Copy FP64 data `which` (SPMV_F64_*) into host out[0..n) (synchronous). */
int spmv_plan_get_f64(spmv_plan_t *plan, int32_t which, double *out, int64_t n);
/* Zero the timing accumulators (per-op event times and host timeline). */
int spmv_plan_reset_times(spmv_plan_t *plan);
/* Profiling of later executions, a bit mask: 1 = per-op GPU timing with HIP
 * events (as SPMV_F_PROFILE; two event records per GPU step and copy), 2 =
 * host timeline (a steady-clock read after each token: where the host waits
 * and for how long); 0 = off.  SPMV_EINVAL outside 0..3. */
int spmv_plan_set_profile(spmv_plan_t *plan, int32_t on);

/* Pinned host buffers owned by the plan: the inbox [n_halo] the caller
 * fills before spmv_exec, and the outbox [n_send] the exec fills. */
int spmv_plan_inbox(spmv_plan_t *plan, double **host_ptr, int64_t *n);
int spmv_plan_outbox(spmv_plan_t *plan, double **host_ptr, int64_t *n);

/* ------------------------------------------------------------ plan space */

/*
 * Validate an operation order and stream map without building a plan
 * (host only).  Same rules and error codes as spmv_plan_create.
 */
int spmv_plan_validate(int32_t nranks, const int32_t *op_order, int32_t n_ops,
                       const int32_t *stream_map, int32_t n_streams);

/*
 * The design space of Sec. III-B/C: every topological order of the SpMV DAG
 * with its Table III tokens, times every stream binding of the GPU vertices
 * up to a stream bijection (Unpack implied before y_R).  Enumerated in a
 * fixed depth-first order (ready tokens ascending by code, streams
 * ascending), so index i names the same plan on every call.
 *   nranks     1 (only START, y_L, END) or > 1 (the full DAG)
 *   n_streams  1..SPMV_MAX_STREAMS
 */
int spmv_plan_space_count(int32_t nranks, int32_t n_streams, int64_t *count);
/* Plan `index` of that space: op_order [SPMV_MAX_OPS] host out, *n_ops out,
 * stream_map [SPMV_N_VERTICES] host out (-1 for CPU vertices). */
int spmv_plan_space_get(int32_t nranks, int32_t n_streams, int64_t index,
                        int32_t *op_order, int32_t *n_ops, int32_t *stream_map);

/* Printable name of a token ("Pack", "CER-after-Pack", ...), the paper's
 * names.  Writes at most cap bytes including the terminator; returns the
 * full length, or SPMV_EINVAL for an unknown token. */
int spmv_op_name(int32_t op, char *buf, int32_t cap);

/* ------------------------------------------------------------ fine-grained */

/*
 * The fine-grained program of a plan's share (multi-rank plans only; see
 * SPMV_PEER).  Its DAG: start -> {Pack[q], y_L, PostRecv[q]};
 * Pack[q] -> PostSend[q] -> WaitSend[q] -> end with CER-after-Pack[q] and
 * CES-b4-PostSend[q] in between (Table III); PostRecv[q] -> WaitRecv[q] ->
 * y_R for every source q; y_L, y_R -> end.  Destinations are the ranks whose
 * send list is not empty, sources the owners of halo entries.
 *
 * spmv_fine_tokens: the DAG's tokens, ascending; tokens [cap] host out,
 *   *n = count (tokens beyond cap are not written).
 * spmv_fine_default: a valid order (receives first, each Pack with its record
 *   on stream 0, y_L and y_R on stream 1); ops / streams [cap] host out.
 * spmv_fine_count: number of fine-grained programs with up to n_streams
 *   streams (orders times canonical stream maps), as a double; SPMV_EINVAL
 *   beyond 40 tokens.
 * spmv_plan_set_fine: make a validated fine-grained order the plan's program
 *   for later execs; op_stream[i] is the stream of position i when it holds
 *   a GPU vertex (ignored otherwise); op_order NULL = the default order.
 *   Errors as spmv_plan_reorder, which returns the plan to coarse orders.
 *   The per-op profile is not kept while a fine-grained order is in force.
 * spmv_fine_validate: the same checks without changing the plan.
 */
int spmv_fine_tokens(const spmv_plan_t *plan, int32_t *tokens, int32_t cap, int32_t *n);
int spmv_fine_default(const spmv_plan_t *plan, int32_t *ops, int32_t *streams, int32_t cap,
                      int32_t *n_ops);
int spmv_fine_count(const spmv_plan_t *plan, int32_t n_streams, double *count);
int spmv_plan_set_fine(spmv_plan_t *plan, const int32_t *op_order, const int32_t *op_stream,
                       int32_t n_ops, int32_t n_streams);
int spmv_fine_validate(const spmv_plan_t *plan, const int32_t *op_order,
                       const int32_t *op_stream, int32_t n_ops, int32_t n_streams);

/* ------------------------------------------------------------ tree search */

/*
 * Monte-Carlo tree search over the same design space (Sec. III-C).  A tree
 * node is a prefix P_k; its children are the tokens spmv_plan_space would
 * place next (same order: token code, then stream).  Each iteration
 *   selection:  from the root, take the child maximising
 *               c * sqrt(ln N / n) + V  (N, n: rollouts through the node and
 *               the child; the first term is -inf for a fully explored
 *               child; V = (t_max - t_min of the child) / (t_max - t_min of
 *               the node) when n >= 2 and N >= 2 and the node's range is not
 *               zero, else 1; the first of equal scores in creation order);
 *               stop at a node that still has an uncreated child;
 *   expansion:  create one uncreated child, drawn at random;
 *   rollout:    complete the program with random children, keep every node
 *               in the tree, benchmark the program;
 *   backprop:   n += 1, t_min = min(t, t_min), t_max = max(t, t_max) on the
 *               path; a node whose children all exist and are fully explored
 *               (or that is complete) is fully explored.
 * Every iteration benchmarks a plan not benchmarked before; the search ends
 * after `iterations` rollouts or when the root is fully explored.
 *
 * Random draws: draw k picks entry r % m of the m candidates, with
 * r = rand[k] when `rand` is given (error SPMV_EINVAL once it runs out),
 * else the k-th output of a 64-bit Mersenne twister seeded with `seed`.
 */
typedef struct {
    int64_t iterations;   /* rollouts; 0 = until the space is exhausted        */
    uint64_t seed;
    double c;             /* exploration constant; 0 = sqrt(2)                 */
    int32_t n_streams;    /* 0 = 2                                             */
    int32_t n_measure;    /* spmv_mcts_run: measurements per plan; 0 = 1       */
    double t_measure;     /* spmv_mcts_run: seconds per measurement; 0 = 0.01  */
    const uint64_t *rand; /* host [n_rand] random draws, or NULL               */
    int64_t n_rand;
    int64_t reserved[4];
} spmv_mcts_opts_t;

/* One node of the final tree (node 0 is the root, the empty prefix). */
typedef struct {
    int32_t parent;       /* -1 for the root                                   */
    int32_t token;        /* token appended to the parent's prefix (-1: root)  */
    int32_t stream;       /* canonical stream of a GPU vertex, else -1         */
    int32_t full;         /* 1 when the subtree is fully explored              */
    int64_t n;            /* rollouts through the node                         */
    double t_min, t_max;  /* over those rollouts (+inf / -inf when n == 0)     */
} spmv_mcts_node_t;

/*
 * Search with a cost table instead of a device: cost[i] is the time of plan
 * i of spmv_plan_space(nranks, n_streams) (n_cost must equal the count).
 * Host only.  Outputs, all host and optional except n_out:
 *   index_out [cap]  plan index of each rollout, in order
 *   time_out  [cap]  its time
 *   *n_out           rollouts made (entries beyond cap are not written)
 *   nodes     [node_cap] the final tree; *n_nodes = nodes in the tree
 */
int spmv_mcts_run_table(int32_t nranks, const double *cost, int64_t n_cost,
                        const spmv_mcts_opts_t *opts, int64_t *index_out, double *time_out,
                        int64_t cap, int64_t *n_out, spmv_mcts_node_t *nodes,
                        int64_t node_cap, int64_t *n_nodes);

/*
 * Search on the device: every rollout re-orders `plans` (spmv_plan_reorder)
 * to the plan and times it with spmv_plan_time(plans, n_plans, x, y,
 * stream, t_measure, n_measure): the time is the median of the n_measure
 * measurements (Sec. III-C3's protocol).  All plans must share nranks.  The
 * plans are left in the order of the last rollout.  Outputs as above.
 */
int spmv_mcts_run(spmv_plan_t *const *plans, int32_t n_plans, const double *const *x,
                  double *const *y, void *stream, const spmv_mcts_opts_t *opts,
                  int64_t *index_out, double *time_out, int64_t cap, int64_t *n_out,
                  spmv_mcts_node_t *nodes, int64_t node_cap, int64_t *n_nodes);

/*
 * Search over the coarse DAG (fine = 0) or the fine-grained DAG of plans[0]'s
 * share (fine = 1), reporting each rollout as an order and its per-position
 * streams: ops_out / streams_out [cap * max_ops] host, rollout k at
 * k * max_ops (max_ops at least the order length).  A rollout is costed by
 * cost(ops, streams, n_ops, user) when cost is given (host only: the plans
 * may be host-only and x / y NULL), else timed on the device as in
 * spmv_mcts_run with the plans switched to the rollout's order
 * (spmv_plan_reorder or spmv_plan_set_fine).  Other outputs as above.
 */
typedef double (*spmv_cost_fn)(const int32_t *ops, const int32_t *streams, int32_t n_ops,
                               void *user);
int spmv_mcts_run_seq(spmv_plan_t *const *plans, int32_t n_plans, const double *const *x,
                      double *const *y, void *stream, int32_t fine, spmv_cost_fn cost,
                      void *user, const spmv_mcts_opts_t *opts, int32_t *ops_out,
                      int32_t *streams_out, int32_t max_ops, double *time_out, int64_t cap,
                      int64_t *n_out, spmv_mcts_node_t *nodes, int64_t node_cap,
                      int64_t *n_nodes);

/* ------------------------------------------------------------ batches */

/*
 * A batch runs the SpMVs of many rank shares (plans, possibly of different
 * matrices and sizes) together: every GPU step of every share goes into
 * grouped persistent kernels whose work lists hold the stream-CSR tiles
 * (column-slab tiles and slab sums included) and gather ranges of the
 * shares, balanced over the blocks longest-first (a slab tile only on its
 * slab's XCD, dealt in share order).  The shares are cut into chunks: per
 * chunk one Pack and one y_L launch, then per chunk Unpack, y_R and the
 * slab sums.  The halo staging becomes copies on the copy streams, chunk by
 * chunk (or copy nodes of a hipGraph).  The paper's host-blocking
 * synchronisations (CER/CES before PostSend, WaitRecv before y_R) become
 * device-side dependencies: a chunk's Pack -> its send copies; a chunk's
 * receive copies -> its Unpack -> its y_R; y_L -> y_R.  One host
 * synchronisation at the end.  A share's y is bit-identical to spmv_exec
 * of its plan: the same tiles are summed by the same device code.
 */
typedef struct spmv_batch spmv_batch_t;   /* opaque */

typedef struct {
    int32_t blocks_per_cu;  /* persistent grid = 256 * blocks_per_cu, 0 = 8  */
    int32_t use_graph;      /* 0 = auto (stream launches when the halo is
                               staged: the graph's copy nodes run one after
                               another and measured 1.3-1.5x slower; the
                               graph otherwise), 1 = hipGraph, 2 = stream
                               launches                                      */
    int32_t xcd_affinity;   /* 0 = auto (on when every chunk holds >= 8
                               shares), 1 = on: the Pack, y_L, Unpack and
                               packed y_R work of share s runs on XCD s mod 8
                               (column-slab tiles always run on their slab's
                               XCD), 2 = off                                 */
    int32_t staging;        /* 0 = halo staged through the plans' pinned
                               mailboxes (the program), 1 = device phase only
                               (no copies: for timing the grouped kernels;
                               y_R then uses whatever the receive buffers
                               hold)                                          */
    int32_t copy_streams;   /* stream launches (use_graph = 2): copy streams
                               per direction, share i's copies on stream
                               i mod copy_streams; 0 = auto (1: concurrent
                               copies of one direction measured slower; the
                               graph chains each direction's copies too),
                               1..4                                           */
    int32_t chunks;         /* the shares cut into this many consecutive
                               chunks (at most n): chunk c's send copies start
                               once its Pack is done, its Unpack / y_R once
                               its receive copies are in, so one chunk's
                               device work runs under the copies of the
                               others, and with XCD affinity a chunk of 8
                               shares keeps one share's Pack and y_L per
                               XCD; 0 = auto (n / 8 chunks, at least 1),
                               1..256                                       */
    int32_t persistent;     /* 0 = auto (2), 1 = persistent blocks: a fixed
                               grid of 256 * blocks_per_cu blocks, each
                               walking its own item list (assigned on the
                               host longest-first, slab tiles dealt in share
                               order), 2 = one block per work item, items
                               that must run on XCD g placed at indices
                               b with b % 8 == g (blocks_per_cu unused)      */
    int32_t reserved[1];
} spmv_batch_opts_t;

typedef struct {
    int32_t n_shares;
    int32_t n_blocks;        /* grid of each persistent grouped kernel      */
    int64_t n_items[3];      /* work items: Pack+y_L, Unpack, y_R (column
                                slab tiles and slab sums included)          */
    int64_t device_bytes;    /* algorithmic device bytes of one batch exec  */
    int64_t host_link_bytes; /* bytes staged over the host link, both ways  */
    int32_t chunk, width;    /* stream-CSR window and load width shared by all */
    int32_t use_graph, xcd_affinity, staging;
    int32_t n_chunks;        /* pipeline chunks of shares                   */
    int32_t persistent;      /* 1: persistent blocks; 0: one block per item  */
    int32_t reserved;
} spmv_batch_info_t;

/*
 * Build a batch over `n` plans (borrowed: they must outlive the batch and are
 * not executed meanwhile).  Every plan must be a device plan whose y_L and
 * y_R use the stream-CSR kernel in packed tiles (y_L with 32- or 16-bit
 * columns, forms 1 and 4; y_R also in column slabs, form 5, with tiles of
 * 256 / lanes rows) with one common chunk and width (the lanes per row may
 * differ).  SPMV_EINVAL otherwise.
 */
int spmv_batch_create(spmv_plan_t *const *plans, int32_t n, const spmv_batch_opts_t *opts,
                      spmv_batch_t **out);

/*
 * Run the batch: for share i, y[i] = (A_i x_i) over its owned rows, with the
 * same halo semantics as spmv_exec (inboxes filled by the caller, outboxes
 * filled on return).  x, y: host arrays of n device pointers (n_loc each).
 * Host-synchronous on return.
 */
int spmv_batch_exec(spmv_batch_t *batch, const double *const *x, double *const *y, void *stream);

int spmv_batch_info(const spmv_batch_t *batch, spmv_batch_info_t *info);
int spmv_batch_destroy(spmv_batch_t *batch);   /* NULL-safe */

/* ------------------------------------------------------------ serving */

/*
 * A server keeps matrices resident on the device and answers y = A x
 * requests with continuous batching: a worker thread admits queued requests
 * while the HBM budget (resident matrices + buffers of requests on the
 * device) and the in-flight limit allow, launches every admitted request
 * that is not yet running as one batch (one grouped stream-CSR launch, with
 * its x/y copies on the batch's stream), keeps up to max_epochs batches on
 * the device at once, and retires them as their events complete.  Requests
 * that arrive while batches run join the next batch.  Each request's y is
 * computed by the same tiles and device code whatever it is batched with,
 * so its bits do not depend on the mix.  mode 1 serves one request at a
 * time (the plain per-call path) with the same kernels.
 */
typedef struct spmv_server spmv_server_t;   /* opaque */

typedef struct {
    int64_t budget_bytes;   /* device bytes for resident matrices and request
                               buffers (0 = 64 GiB)                          */
    int32_t max_inflight;   /* requests on the device at once (0 = 256)      */
    int32_t max_epochs;     /* batches on the device at once (0 = 4)         */
    int32_t max_batch;      /* requests per batch (0 = 64)                   */
    int32_t chunk;          /* stream-CSR chunk of resident matrices (0 = 8) */
    int32_t mode;           /* 0 = continuous batching, 1 = plain per-call   */
    int32_t reserved[3];
} spmv_server_opts_t;

typedef struct {
    int64_t submitted, completed, batches;
    int64_t resident_bytes;     /* matrices                                  */
    int64_t peak_inflight_bytes;/* request buffers on the device, peak       */
    int64_t arena_bytes;        /* request-buffer arena                      */
    int32_t peak_inflight;      /* requests on the device, peak              */
    int32_t n_matrices;
    double mean_batch;          /* requests per batch                        */
} spmv_server_stats_t;

int spmv_server_create(const spmv_server_opts_t *opts, spmv_server_t **out);
/* Upload a matrix (square, host CSR, borrowed) as a resident single-rank
 * plan; *id receives its index.  SPMV_EBUDGET if it does not fit the budget
 * (leaving room for one request on it).  Only before spmv_server_start. */
int spmv_server_add_matrix(spmv_server_t *srv, const spmv_csr_t *csr, int32_t *id);
/* Start the worker thread (after adding the matrices). */
int spmv_server_start(spmv_server_t *srv);
/* Queue y_host = A[matrix] x_host.  x_host / y_host: host buffers of n rows
 * (pinned memory for asynchronous copies), valid until completion.
 * Non-blocking.  SPMV_EBUDGET if the request could never fit the budget. */
int spmv_server_submit(spmv_server_t *srv, int32_t matrix, const double *x_host, double *y_host,
                       int64_t tag);
/* Completed requests since the last poll: up to cap (tag, latency seconds =
 * completion - submission) pairs; *n receives the count.  Non-blocking. */
int spmv_server_poll(spmv_server_t *srv, int64_t *tags, double *latency_s, int32_t cap,
                     int32_t *n);
/* Block until every submitted request has completed. */
int spmv_server_drain(spmv_server_t *srv);
/* Replay an arrival trace: request i is submitted at arrival_s[i] seconds
 * after the call starts (ascending), for matrix[i] with x_host[i] /
 * y_host[i]; returns when all completed, latency_s[i] = completion -
 * arrival.  *wall_s receives the time from the first arrival to the last
 * completion. */
int spmv_server_run_trace(spmv_server_t *srv, int64_t n, const int32_t *matrix,
                          const double *arrival_s, const double *const *x_host,
                          double *const *y_host, double *latency_s, double *wall_s);
int spmv_server_stats(spmv_server_t *srv, spmv_server_stats_t *stats);
int spmv_server_destroy(spmv_server_t *srv);   /* drains, stops, frees; NULL-safe */

/* ------------------------------------------------------------ no allocation */

/* Bytes of the library's fixed per-device scratch array (64 MiB). */
#define SPMV_STATIC_SCRATCH_BYTES (64ll << 20)

/*
 * spmv_exec for callers that cannot allocate device memory around their
 * calls (a tight serving loop, a harness that forbids it): the same exec,
 * with the same arguments, results and errors as spmv_exec, except that
 * the per-exec intermediate data (send buffer, receive buffer, unpacked
 * halo, remote partial sums, column-slab partial sums) lives in one fixed
 * device array of the library instead of the plan's own buffers.  The call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *
 * The array holds SPMV_STATIC_SCRATCH_BYTES on every GPU the library runs
 * on, until the process ends; its device address is looked up on the first
 * call on a device.  A plan whose exec needs more (8 bytes per send entry
 * and per halo entry, 8 more per halo entry when Unpack is not fused, 8 per
 * remote row, 64 per remote row in column slabs, each piece rounded up to
 * 256 bytes) is refused with SPMV_EINVAL before anything runs.  Every call
 * on one GPU uses the same array and leaves its last contents there (each
 * piece is written in full before it is read, so no call depends on them):
 * calls that overlap on one GPU (from several host threads) race and must
 * not be issued.  The call is host-synchronous like spmv_exec, so calls
 * from one thread never overlap.  spmv_plan_get_f64 keeps describing the
 * plan's own buffers (the last spmv_exec), not the static array; the
 * outbox receives the send buffer as with spmv_exec.
 */
int spmv_exec_static(spmv_plan_t *plan, const double *x_local, double *y_local, void *stream);
/* SPMV_STATIC_SCRATCH_BYTES, as compiled into the library. */
int64_t spmv_static_scratch_bytes(void);

/* ------------------------------------------------------------ measurement */

/*
 * HBM probe: the achievable-bandwidth yardstick for the SpMV kernels.
 *   mode 0  read every byte of src once (16-byte loads) and write one partial
 *           sum per block to dst (device, >= `blocks` doubles)
 *   mode 1  copy `bytes` from src to dst (device, non-overlapping)
 *   mode 2  gather: spmv_gathers_per_probe_block() random 8-byte loads per
 *           block at hashed indices, block b inside window b mod 8 of src
 *           (src cut into 8 equal windows of bytes / 64 doubles: the x
 *           gathers of the column-slab remote product, each XCD's from its
 *           own L2), one partial sum per block to dst
 *   mode 3  the same gathers over all of src (a halo larger than the L2)
 * bytes: a multiple of 16 (modes 2, 3: at most 2^32 - 1 doubles); blocks:
 * grid size, 0 = 2048.  Asynchronous on `stream`; the caller times it (e.g.
 * with events around repeated calls).
 */
int spmv_hbm_probe(int32_t mode, const void *src, void *dst, int64_t bytes, int32_t blocks,
                   void *stream);
/* Gathers one block of the gather probe (modes 2, 3) makes. */
int64_t spmv_gathers_per_probe_block(void);

/* ------------------------------------------------------------ misc */

const char *spmv_last_error(void);
const char *spmv_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPMV_H */
