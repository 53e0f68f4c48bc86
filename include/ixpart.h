/*
 * ixpart.h -- C ABI of the MI355X (gfx950) filter-partition library.
 *
 * The library computes, on one AMD Instinct MI355X, the data-parallel programs
 * whose index arrays the paper "Verifying Properties of Index Arrays in a
 * Purely-Functional Data-Parallel Language" reasons about:
 *   - partition2 (Section 2.1, figure "Running Examples"): a stable two-way
 *     partition built from map (the predicate), scan (+) of the flags, an
 *     index map and a scatter;
 *   - filter (FiltPart with a filtering predicate, Section 2.3 and Section 6);
 *   - the v-way partition (FiltPart with v predicates, Section 2.3;
 *     partition3 of Section 6);
 *   - partition2L / filter_seg (Section 6, "Segmented operations"): the same
 *     applied to every row of a jagged array given by its shape, rows may be
 *     empty;
 *   - scatter (Section 2.1) restricted to injective index arrays, and its
 *     inverse, a gather;
 *   - run-time checkers of the array properties Range, Monotonic, Inj, Bij and
 *     FiltPart (Section 2.3, figure "Array Properties");
 *   - the dynamically verified scatter and the reduce-by-index with min that
 *     the evaluation compares the statically verified path against
 *     (Section 6).
 *
 * Conventions common to every entry point
 *   - Pointers named d_* or documented as "device" are device pointers
 *     (hipMalloc / torch CUDA tensors); the caller owns every buffer.  Other
 *     pointers (ixp_pred, ixp_prop_args, ixp_tuning) are host pointers read
 *     during the call only.
 *   - Device buffers must be aligned to their element size.  Buffers aligned
 *     to 16 bytes take the vector-load path; others are still correct.
 *   - `stream` is a hipStream_t passed as void* (NULL = null stream).  Every
 *     call only enqueues work on `stream`: no host synchronisation, no
 *     allocation, no hipMemset -- except the functions documented as
 *     "blocking" (autotuning, graph creation, error read-back).
 *   - Argument errors are detected on the host before anything is enqueued and
 *     reported as a negative status; a failed kernel launch returns IXP_EHIP.
 *     No C++ exception crosses this interface.
 *   - Workspaces: query the size, allocate device memory of at least that many
 *     bytes, pass it in.  Its contents need no initialisation; a workspace may
 *     not be shared by calls that can run concurrently.
 */
#ifndef IXPART_H
#define IXPART_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
enum {
    IXP_OK = 0,
    IXP_EINVAL = -1,        /* bad argument: null pointer, negative size, ... */
    IXP_ENOMEM = -2,        /* host allocation failed (graph objects only)    */
    IXP_EHIP = -3,          /* a HIP runtime call or kernel launch failed     */
    IXP_EUNSUPPORTED = -4,  /* valid request this build does not implement    */
    IXP_EWORKSPACE = -5,    /* workspace missing or smaller than required     */
    IXP_EDEVICE = -6,       /* a kernel reported an error in the workspace    */
    IXP_ETOOLARGE = -7      /* n exceeds a fixed capacity (static scratch)    */
};
const char *ixp_status_str(int status);

/* ---- element types, predicates, modes ------------------------------------ */
enum { IXP_I32 = 0, IXP_I64 = 1, IXP_F32 = 2, IXP_U8 = 3 };

/* The predicate p mapped over the keys (Section 2.1: cs = map p xs).
 *   IXP_PRED_MOD_EQ: keys I32; p(x) = (x mod d == r) with the floor modulus
 *                    (result in [0,d)); 1 <= d < 2^32.
 *   IXP_PRED_LT:     keys F32; p(x) = (x < s), one IEEE single comparison,
 *                    NaN gives false.
 *   IXP_PRED_FLAGS:  keys I32 or F32 (moved as bits); p(i) = flags[i] != 0,
 *                    `flags` a device u8 array of length n (partition2L's csL;
 *                    NULL allowed when n == 0).
 * Predicates of the row number k (segmented calls only; Section 1: segmented
 * partitioning by predicates that depend on the segment number):
 *   IXP_PRED_LT_ROW:  keys F32; p_k(x) = (x < row_s[k]), `row_s` a device
 *                     f32 array of length m;
 *   IXP_PRED_MOD_ROW: keys I32; p_k(x) = (x mod d == k mod d), floor moduli,
 *                     1 <= d < 2^32. */
enum { IXP_PRED_MOD_EQ = 0, IXP_PRED_LT = 1, IXP_PRED_FLAGS = 2,
       IXP_PRED_LT_ROW = 3, IXP_PRED_MOD_ROW = 4 };
typedef struct {
    int32_t kind;
    int32_t reserved0;
    int64_t d;
    int64_t r;
    float s;
    int32_t reserved1;
    const uint8_t *flags;   /* device */
    const float *row_s;     /* device, IXP_PRED_LT_ROW */
} ixp_pred;

/* IXP_MODE_PARTITION: FiltPart with p^f = true and partition predicate p --
 *   partition2: trues first, falses after, both in input order.
 * IXP_MODE_FILTER: FiltPart with p^f = p and no partition -- filter: only the
 *   trues are kept, in input order; dropped elements get index -1. */
enum { IXP_MODE_PARTITION = 0, IXP_MODE_FILTER = 1 };

/* ---- flat partition (partition2 / filter) -------------------------------- */

/* Bytes of workspace ixp_partition needs for n elements. */
size_t ixp_partition_workspace(int64_t n);

/* Stable partition of keys[0..n) by `pred` (Section 2.1, partition2):
 *   out_idx[i]  = destination of element i, the scatter index array whose
 *                 InvFiltPart property the paper states:
 *                   PARTITION: c_i ? #trues before i : T + #falses before i
 *                   FILTER:    c_i ? #trues before i : -1
 *   out_keys    = scatter of the keys by out_idx (length n in PARTITION mode,
 *                 T in FILTER mode; positions >= T untouched in FILTER mode);
 *   *d_split    = T, the number of trues (partition2's num_true), int64.
 * key_t: IXP_I32 or IXP_F32 (see ixp_pred); idx_t: IXP_I32 (needs n < 2^31)
 * or IXP_I64.  out_keys and out_idx may each be NULL (not produced); d_split
 * is required.  n == 0 is valid and writes T = 0.
 * Enqueues 2-3 kernels on `stream`; capturable into a HIP graph. */
int ixp_partition(const void *keys, int32_t key_t, int64_t n,
                  const ixp_pred *pred, int32_t mode, void *out_keys,
                  void *out_idx, int32_t idx_t, int64_t *d_split, void *ws,
                  size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * operation, arguments and results as ixp_partition, with the workspace
 * replaced by a scratch array of IXP_NOALLOC_SCRATCH_BYTES bytes that the
 * library holds in device memory on every GPU it runs on (from the loading of
 * its code object until the process ends).  It calls no hipMalloc, hipFree or
 * other allocating routine; the first call on a device looks up that device's
 * copy of the array once.
 *   n above IXP_NOALLOC_MAX_N (2,180,907,008 elements: 532,448 descriptors of
 *   4096-element tiles) returns IXP_ETOOLARGE and enqueues nothing; every
 *   other argument error is reported as by ixp_partition.
 * All calls on one GPU share that GPU's scratch: calls that may overlap in
 * time on one GPU (different streams, or host threads without ordering) race
 * and give undefined results; calls ordered on one stream are safe.  The
 * scratch keeps the last call's contents, and each call's kernels clear what
 * they read before use.  A look-back that gave up (filter mode) is recorded
 * in the scratch, where ixp_read_error cannot reach it. */
#define IXP_NOALLOC_SCRATCH_BYTES ((size_t)4325376)
#define IXP_NOALLOC_MAX_N ((int64_t)2180907008)
int ixp_partition_noalloc(const void *keys, int32_t key_t, int64_t n,
                          const ixp_pred *pred, int32_t mode, void *out_keys,
                          void *out_idx, int32_t idx_t, int64_t *d_split,
                          void *stream);

/* ---- v-way partition (partition3) ----------------------------------------- */

/* The class c(i) in [0, v) of element i, 2 <= v <= 4: the v pairwise exclusive
 * predicates p_1..p_v of FiltPart (Section 2.3), p_{c+1} holding for class c
 * and p_v = not (p_1 or ... or p_{v-1}).
 *   IXP_CLASS_MOD:    int32 keys, c = floor-mod(key, v);
 *   IXP_CLASS_THRESH: f32 keys, thresholds s[0] <= ... <= s[v-2]: class h
 *                     for s[h-1] <= x < s[h] (class 0: x < s[0]), the last
 *                     class for x >= s[v-2] and for NaN;
 *   IXP_CLASS_BYTES:  c = min(classes[i], v - 1), `classes` a device u8[n]
 *                     (4-byte aligned; NULL allowed when n == 0). */
enum { IXP_CLASS_MOD = 0, IXP_CLASS_THRESH = 1, IXP_CLASS_BYTES = 2 };

typedef struct {
    int32_t kind;
    int32_t v;
    float s[3];
    int32_t reserved;
    const uint8_t *classes;   /* device */
} ixp_classes;

size_t ixp_partition_v_workspace(int64_t n);

/* Stable v-way partition of keys[0..n) (FiltPart with v predicates and no
 * filtering, Section 2.3; partition3 of Section 6 is v = 3): class 0 first,
 * then class 1, ..., each class in input order.
 *   out_idx[i]   = N_0 + ... + N_{c(i)-1} + #earlier elements of class c(i);
 *   out_keys     = scatter of the keys by out_idx (length n);
 *   d_counts[c]  = N_c, the size of class c (device int64[v]).
 * key_t IXP_I32 or IXP_F32 (moved as bits); idx_t IXP_I32 (n < 2^31) or
 * IXP_I64.  out_keys / out_idx may be NULL.  Alignment (else IXP_EINVAL): keys
 * 16 bytes, out_idx 4 indices, out_keys 4 bytes.  Unsorted thresholds are
 * IXP_EINVAL.  Enqueues 3 kernels; capturable into a HIP graph. */
int ixp_partition_v(const void *keys, int32_t key_t, int64_t n,
                    const ixp_classes *cls, void *out_keys, void *out_idx,
                    int32_t idx_t, int64_t *d_counts, void *ws,
                    size_t ws_bytes, void *stream);

/* ---- segmented partition (partition2L / filter_seg) ----------------------- */

/* Tile shape of the segmented kernels: `block` threads (256, 512 or 1024)
 * each holding `rows` x 4 elements (rows in {2,4,8}, tile <= 16384); a tile
 * is block*rows*4 elements, and every row is cut into work items of at most
 * one tile.  `wgs_per_cu` (1..64, 0 = as many as fit) sizes the grid of the
 * main kernel: workgroup w takes items w, w + grid, w + 2*grid, ...
 * `row_sync` says how, in PARTITION mode, a row of 2..256 items learns its
 * true count T_k (rows of more items always take the counting pass):
 *   IXP_ROW_SYNC_WAIT  (3) inside the main kernel: each item publishes its
 *                      own count and waits, for a bounded number of polls,
 *                      for those of the row's other items; an item still
 *                      unpublished then is counted from its keys by the
 *                      waiting workgroup, so the wait always ends and the
 *                      result does not depend on timing.  It pays when the
 *                      grid is oversubscribed (the hardware then starts a
 *                      row's items back to back); with persistent grids the
 *                      workgroups drift apart and the waits grow;
 *   IXP_ROW_SYNC_COUNT (1) a separate counting pass reads the row first;
 *   IXP_ROW_SYNC_AUTO  (0) WAIT with 16 or more workgroups per CU, else COUNT;
 *   IXP_ROW_SYNC_NOWAIT(2) as WAIT with no polling: every sibling not yet
 *                      published is counted by the waiting workgroup (the
 *                      fallback of WAIT, made the rule; for tests).
 * A NULL tuning pointer selects the default: 256 x 4, 64 workgroups per CU,
 * AUTO. */
enum { IXP_ROW_SYNC_AUTO = 0, IXP_ROW_SYNC_COUNT = 1, IXP_ROW_SYNC_NOWAIT = 2, IXP_ROW_SYNC_WAIT = 3 };
typedef struct {
    int32_t block;
    int32_t rows;
    int32_t wgs_per_cu;
    int32_t row_sync;
} ixp_tuning;

size_t ixp_segmented_workspace(int64_t n, int64_t m, const ixp_tuning *tune);

/* partition2 applied to each row of a jagged array (Section 6, partition2L).
 * d_shape: device int64[m], row sizes (>= 0, empty rows allowed, sum = n).
 * Row k covers [o_k, o_k + shape[k]) with o_k the sum of the earlier sizes.
 *   PARTITION: out_idx[i] = o_k + (c_i ? #trues before i in row k
 *                                       : T_k + #falses before i in row k),
 *              out_keys   = every row partitioned in place of the row;
 *   FILTER:    kept elements of all rows packed row after row (filter_seg),
 *              out_idx[i] = -1 for dropped elements.
 *   d_seg_split[k] = T_k, the number of trues of row k (device int64[m]).
 *   d_flags_out (nullable, device u8[n]) = the segment descriptor: 1 at the
 *              first element of every non-empty row, 0 elsewhere (mkSgmDescr
 *              applied to a row of ones, Section 2.1).
 * out_keys, out_idx, d_seg_split and d_flags_out may each be NULL (not
 * produced); keys may be NULL when the predicate is IXP_PRED_FLAGS and
 * out_keys is NULL.
 * A negative size or a size sum different from n is detected on the device:
 * the call then writes no output and ixp_read_error() on the same workspace
 * reports IXP_EINVAL.  Enqueues 6 kernels (shape scan, item records, counts
 * of the multi-item rows that the main kernel does not synchronise itself,
 * item scan, item bases, main), all stream-ordered with no host
 * synchronisation: capturable into a HIP graph.  Under IXP_ROW_SYNC_WAIT the
 * main kernel's workgroups wait on one another's published counts; the wait
 * is bounded, so no workgroup depends on another being resident.
 * Alignment (else IXP_EINVAL): keys and ws 16 bytes, out_idx 4 indices,
 * out_keys, d_flags_out and a flag predicate's array 4 bytes. */
int ixp_segmented_partition(const void *keys, int32_t key_t, int64_t n,
                            const int64_t *d_shape, int64_t m,
                            const ixp_pred *pred, int32_t mode, void *out_keys,
                            void *out_idx, int32_t idx_t, int64_t *d_seg_split,
                            uint8_t *d_flags_out, const ixp_tuning *tune,
                            void *ws, size_t ws_bytes, void *stream);

/* The segment helpers of Section 2.1 (figure "Running Examples", right) as
 * device outputs, for rows of sizes d_shape[0..m) (>= 0, summing to n; a bad
 * shape is reported by ixp_read_error as IXP_EINVAL and nothing is written):
 *   ixp_mk_ii:        out[i] = k for every i of row k (mkII), out_t IXP_I32
 *                     or IXP_I64;
 *   ixp_mk_sgm_descr: d_out[o_k] = d_xs[k] for every non-empty row k, 0 at
 *                     every other position (mkSgmDescr), int64.
 * Workspace: ixp_mk_ii_workspace(n, m) bytes, 16-byte aligned.  3 kernels. */
size_t ixp_mk_ii_workspace(int64_t n, int64_t m);
int ixp_mk_ii(const int64_t *d_shape, int64_t m, int64_t n, void *out,
              int32_t out_t, void *ws, size_t ws_bytes, void *stream);
int ixp_mk_sgm_descr(const int64_t *d_shape, int64_t m, int64_t n,
                     const int64_t *d_xs, int64_t *d_out, void *ws,
                     size_t ws_bytes, void *stream);

/* sgmSum (Section 2.1, figure "Running Examples", right): d_out[i] = the
 * inclusive scan of d_xs under (fx, vx) (+) (fy, vy) = (fx || fy, fy ? vy :
 * vx + vy), i.e. the sum of d_xs over [last j <= i with d_flags[j] != 0, i]
 * (from 0 if no such j).  int64 values (wrapping on overflow), u8 flags.
 * Workspace: ixp_sgm_sum_workspace(n) bytes, 8-byte aligned.  3 kernels
 * (chunk aggregates, their scan, a rescan of each chunk). */
size_t ixp_sgm_sum_workspace(int64_t n);
int ixp_sgm_sum(const uint8_t *d_flags, const int64_t *d_xs, int64_t n,
                int64_t *d_out, void *ws, size_t ws_bytes, void *stream);

/* Blocking: times every candidate tiling (tile shape, grid and, in PARTITION
 * mode, row sync WAIT or COUNT) on the given arguments (which it overwrites)
 * and stores the fastest in *best (and its time in *best_ms). */
int ixp_tune_segmented(const void *keys, int32_t key_t, int64_t n,
                       const int64_t *d_shape, int64_t m, const ixp_pred *pred,
                       int32_t mode, void *out_keys, void *out_idx,
                       int32_t idx_t, int64_t *d_seg_split,
                       uint8_t *d_flags_out, void *ws, size_t ws_bytes,
                       int32_t reps, ixp_tuning *best, float *best_ms,
                       void *stream);

/* HIP-graph form: blocking creation captures one ixp_segmented_partition call
 * (all its kernels) into an instantiated graph; ixp_graph_launch replays it on
 * `stream` with the same pointers and sizes (contents may change between
 * launches).  Destroy with ixp_graph_destroy. */
typedef struct ixp_graph_s *ixp_graph;
int ixp_segmented_graph_create(ixp_graph *out, const void *keys, int32_t key_t,
                               int64_t n, const int64_t *d_shape, int64_t m,
                               const ixp_pred *pred, int32_t mode,
                               void *out_keys, void *out_idx, int32_t idx_t,
                               int64_t *d_seg_split, uint8_t *d_flags_out,
                               const ixp_tuning *tune, void *ws,
                               size_t ws_bytes);
int ixp_graph_launch(ixp_graph g, void *stream);
int ixp_graph_destroy(ixp_graph g);

/* Blocking: synchronises `stream` and returns IXP_OK, or the error a kernel
 * recorded in the workspace of the last call that used `ws` (IXP_EINVAL for a
 * bad shape array, IXP_EDEVICE for an exhausted wait); then clears it. */
int ixp_read_error(const void *ws, void *stream);

/* ---- scatter / gather of rows (Section 2.1 scatter; Bij inverse) ----------- */

/* dst[idx[i]] := vals[i] (rows of row_bytes bytes) for i in [0,m) with
 * 0 <= idx[i] < n_dst; other indices are ignored, as scatter ignores
 * out-of-bounds writes.  Precondition (not checked): Inj idx [0,n_dst), so no
 * two rows race (scatter's idempotence requirement).  row_bytes must be a
 * multiple of 4; multiples of 16 with 16-byte aligned buffers use vector
 * stores.  Plain stores, no atomics. */
int ixp_scatter_inj(void *dst, int64_t n_dst, const void *idx, int32_t idx_t,
                    const void *vals, int64_t m, int64_t row_bytes,
                    void *stream);

/* dst[i] := src[idx[i]] for i in [0,m) (rows of row_bytes bytes).  An index
 * outside [0,n_src) produces a zero row and, if d_err is not NULL, sets
 * *d_err = 1 (device int32); the caller zeroes *d_err. */
int ixp_gather(void *dst, const void *src, int64_t n_src, const void *idx,
               int32_t idx_t, int64_t m, int64_t row_bytes, int32_t *d_err,
               void *stream);

/* ---- property checkers (Section 2.3, figure "Array Properties") ----------- */
enum {
    IXP_RANGE = 1,    /* lo <= X[i] < hi for all i                           */
    IXP_MONO = 2,     /* X[i-1] op X[i] for 1 <= i < n                       */
    IXP_INJ = 4,      /* no repeated value among entries inside [lo,hi)      */
    IXP_BIJ = 8,      /* Inj, in-Rcd values inside Img, count = |Img|        */
    IXP_FILTPART = 16 /* outputs of a flat partition are a filter-partition   */
};
enum { IXP_MONO_LE = 0, IXP_MONO_LT = 1, IXP_MONO_GE = 2, IXP_MONO_GT = 3 };

/* One verdict per property, written to device memory:
 *   holds = 1/0; first_violation = -1 if it holds, else the least failing
 *   index (see the per-property definitions below); aux = a value naming the
 *   failure.
 *   RANGE: first i with X[i] outside [lo,hi); aux = X[i].
 *   MONO:  first i >= 1 with !(X[i-1] op X[i]); aux = 0.
 *   INJ:   first i with X[i] in [lo,hi) equal to some earlier X[j]; aux = X[i].
 *   BIJ:   first i with X[i] in [lo,hi) repeated earlier or outside
 *          [img_lo,img_hi) (aux = X[i]); failing only on the count:
 *          first_violation = n, aux = least value of Img not attained.
 *   FILTPART: X = the partitioned keys (fp_src, key type fp_key_t), Y =
 *          fp_dst (n entries, as ixp_partition writes them; FILTER compares
 *          the first split), Z = x (the index array), split = *fp_split,
 *          pred / mode as given to ixp_partition.  aux = OR of failing
 *          sub-checks: 1 split != #trues (#kept); 2 Z not a bijection onto
 *          [0,n) (FILTER: kept Z not injective into [0,split), or a dropped
 *          Z inside [0,split)); 4 class order (Z[i] < split iff p, PARTITION
 *          only); 8 Z not strictly increasing inside a class (FILTER: among
 *          kept elements); 16 Y[Z[i]] != X[i] bitwise.  first_violation = the
 *          least index failing one of 2..16, n if only 1 fails.
 * Intervals are half-open.  Inj and Bij need a workspace of about 4.25 bytes
 * per value of Rcd [lo,hi) (two bitmaps and a first-index table), plus 4
 * bytes per element when n >= 2^16; Rcd may span at most 2^36 values. */
typedef struct {
    int32_t holds;
    int32_t reserved;
    int64_t first_violation;
    int64_t aux;
} ixp_verdict;

typedef struct {
    int64_t lo, hi;            /* RANGE interval; INJ/BIJ restricted co-domain */
    int64_t img_lo, img_hi;    /* BIJ image, inside [lo,hi)                     */
    int32_t mono_op;           /* IXP_MONO_*                                    */
    int32_t fp_mode;           /* IXP_MODE_* of the checked partition           */
    const void *fp_src;        /* device keys that were partitioned             */
    const void *fp_dst;        /* device partitioned keys                       */
    int32_t fp_key_t;          /* IXP_I32 or IXP_F32                            */
    int32_t reserved;
    ixp_pred fp_pred;          /* the partition predicate                      */
    const int64_t *fp_split;   /* device int64, the split point                 */
} ixp_prop_args;

size_t ixp_check_props_workspace(int64_t n, uint32_t mask,
                                 const ixp_prop_args *a);

/* Checks the properties selected by `mask` (IXP_* bits) on the device array
 * x[0..n) of type x_t (IXP_I32 or IXP_I64; x 16-byte aligned, the workspace
 * 256-byte aligned) and writes d_out[b] for every bit b
 * in 0..4 (unselected properties get holds = 1, first_violation = -1).
 * Verdicts are deterministic: independent of scheduling and bit-exact with
 * the definitions above. */
int ixp_check_props(const void *x, int32_t x_t, int64_t n, uint32_t mask,
                    const ixp_prop_args *a, ixp_verdict *d_out, void *ws,
                    size_t ws_bytes, void *stream);

/* ---- dynamic verification of scatter, reduce-by-index (Section 6) --------- */

/* Reduce-by-index with min (the `hist i64.min` of get_smallest_pairs,
 * Section 6): d_dst[0..n_dst) := neutral, then for every i < m with
 * 0 <= idx[i] < n_dst, d_dst[idx[i]] := min(d_dst[idx[i]], vals[i]); a NULL
 * `vals` stands for vals[i] = i.  Other indices are ignored.  Device int64
 * arrays (vals nullable), idx of type idx_t.  Deterministic (min is
 * order-independent); device atomics, 2 kernels. */
int ixp_hist_min(int64_t *d_dst, int64_t n_dst, int64_t neutral,
                 const void *idx, int32_t idx_t, const int64_t *vals,
                 int64_t m, void *stream);

/* d_flags[k] := 1 if 0 <= idx[k] < n_hist and d_hist[idx[k]] == vals[k],
 * else 0, for k < m: the step of get_smallest_pairs (Sections 5.4 and 6)
 * that keeps an entry whose value is the minimum recorded at its endpoint,
 * d_hist being an ixp_hist_min result.  The flags
 * feed a filter with IXP_PRED_FLAGS.  d_flags 4-byte aligned; int64 hist and
 * vals; idx of type idx_t.  1 kernel. */
int ixp_match_min(uint8_t *d_flags, const int64_t *d_hist, int64_t n_hist,
                  const void *idx, int32_t idx_t, const int64_t *vals,
                  int64_t m, void *stream);

size_t ixp_scatter_checked_workspace(int64_t n_dst);

/* The dynamically verified scatter of the evaluation's Base variant
 * (Section 6, table "tab:eval": scatter into a zeroed array, checked at run
 * time with a reduce-by-index of atomic minima):
 *   dst[0..n_dst) := 0 (elements of elem_bytes = 4 or 8 bytes);
 *   win[v] := the least i with idx[i] == v (ixp_hist_min over iota);
 *   dst[v] := vals[win[v]] for every written location v;
 *   *d_out  := Inj of idx over [0, n_dst): holds iff no in-bounds location is
 *             written twice; first_violation = the least i whose location an
 *             earlier i also writes, aux = idx[first_violation].
 * Out-of-bounds indices are ignored.  Workspace: ixp_scatter_checked_workspace
 * bytes, 256-byte aligned (8 bytes per location).  4 kernels. */
int ixp_scatter_checked(void *dst, int64_t n_dst, const void *idx,
                        int32_t idx_t, const void *vals, int64_t m,
                        int64_t elem_bytes, ixp_verdict *d_out, void *ws,
                        size_t ws_bytes, void *stream);

/* d[0..bytes) := 0 with a kernel (no hipMemset, so it may be captured into
 * a HIP graph): the initialisation `replicate n 0` of a scattered array. */
int ixp_zero(void *d, size_t bytes, void *stream);

/* ---- kernel timing ------------------------------------------------------------ */
/* While enabled, every kernel the library enqueues (outside HIP-graph capture)
 * is bracketed by two HIP events recorded on its own stream.  ixp_profile_read
 * is blocking: it waits for the recorded events, writes up to `max` per-kernel
 * summaries (name, launches, total milliseconds), stores the number of
 * distinct kernels in *count, and clears the records. */
typedef struct {
    char name[64];
    int64_t launches;
    double total_ms;
} ixp_kernel_stat;
int ixp_profile_enable(int on);
int ixp_profile_read(ixp_kernel_stat *out, int max, int *count);

/* ---- device information ----------------------------------------------------- */
/* Number of compute units of the current device (cached), or a negative status. */
int ixp_device_cus(void);

#ifdef __cplusplus
}
#endif
#endif /* IXPART_H */
