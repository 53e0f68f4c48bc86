/*
 * ixoracle.c -- plain, sequential CPU oracle for the filter-partition path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no header, helper, table or
 * constant with the HIP implementation.
 *
 * Every result computed here has a plain definition, and each routine is
 * that definition written out as a sequential loop, with no blocking, fusion
 * or reordering:
 *   - map and scatter semantics: Section 2.1 (combinator types and the
 *     imperative meaning of scatter);
 *   - partition2 / filter (the stable two-way partition and the order-keeping
 *     filter), sgmSum, mkSgmDescr, mkII: Section 2.1;
 *   - partition2L (partition2 of every row of a jagged array): Section 6,
 *     "Segmented operations";
 *   - the properties Range, Monotonic, Inj, Bij, FiltPart / InvFiltPart:
 *     Section 2.3, figure "Array Properties" and the prose after it.
 * Readings taken where the paper is ambiguous are listed beside the code that
 * takes them.  Integer work only, except the f32 predicate x < s, which is a
 * single IEEE single-precision comparison (the paper's benchmark arrays are
 * f32, Section 6).
 *
 * Return value convention: 0 on success, -1 on invalid arguments,
 * -2 on allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { IXO_I32 = 0, IXO_I64 = 1, IXO_F32 = 2 };
enum { IXO_PRED_MOD_EQ = 0, IXO_PRED_LT = 1, IXO_PRED_FLAGS = 2 };
enum { IXO_MODE_PARTITION = 0, IXO_MODE_FILTER = 1 };
enum { IXO_MONO_LE = 0, IXO_MONO_LT = 1, IXO_MONO_GE = 2, IXO_MONO_GT = 3 };

/* ------------------------------------------------------------------------ */
/* The predicate p, applied to every element by a map (Section 2.1).       */
/* MOD_EQ: floor-modulus of an integer key by d equals r (d > 0).  The paper */
/* does not fix the sign convention of %; floor-mod (result in [0,d)) is    */
/* the reading taken.  LT: f32 key < s, IEEE comparison (NaN gives false).  */
/* FLAGS: a caller-supplied boolean array (partition2L's csL input).        */
/* ------------------------------------------------------------------------ */
static int64_t floor_mod(int64_t a, int64_t d) {
    int64_t r = a % d;
    if (r < 0) r += d;
    return r;
}

static int valid_key_t(int key_t) {
    return key_t == IXO_I32 || key_t == IXO_I64 || key_t == IXO_F32;
}

static int64_t key_bytes(int key_t) { return key_t == IXO_I64 ? 8 : 4; }

int ixo_map_pred(const void *xs, int key_t, int64_t n, int pred_kind,
                 int64_t d, int64_t r, float s, const uint8_t *flags_in,
                 uint8_t *cs) {
    if (n < 0 || (n > 0 && !cs)) return -1;
    if (pred_kind == IXO_PRED_MOD_EQ) {
        if (d <= 0 || (n > 0 && !xs)) return -1;
        if (key_t != IXO_I32 && key_t != IXO_I64) return -1;
        for (int64_t i = 0; i < n; i++) {
            int64_t x = key_t == IXO_I32 ? (int64_t)((const int32_t *)xs)[i]
                                         : ((const int64_t *)xs)[i];
            cs[i] = floor_mod(x, d) == r;
        }
    } else if (pred_kind == IXO_PRED_LT) {
        if (key_t != IXO_F32 || (n > 0 && !xs)) return -1;
        for (int64_t i = 0; i < n; i++) {
            float x = ((const float *)xs)[i];
            cs[i] = x < s;
        }
    } else if (pred_kind == IXO_PRED_FLAGS) {
        if (n > 0 && !flags_in) return -1;
        for (int64_t i = 0; i < n; i++) cs[i] = flags_in[i] != 0;
    } else {
        return -1;
    }
    return 0;
}

/* scatter dst is vs: for i in 0..m-1, if 0 <= is[i] < len(dst) then
 * dst[is[i]] := vs[i] (Section 2.1).  Writes outside dst are the ones
 * ignored: the bound is the length of dst (the type of scatter gives dst
 * length n; a bound of m is read as a slip).  Elements are moved as raw
 * bytes. */
int ixo_scatter(void *dst, int64_t n_dst, const int64_t *is, const void *vs,
                int64_t m, int64_t elem_bytes) {
    if (n_dst < 0 || m < 0 || elem_bytes <= 0) return -1;
    if (m > 0 && (!is || !vs)) return -1;
    for (int64_t i = 0; i < m; i++) {
        if (0 <= is[i] && is[i] < n_dst)
            memcpy((char *)dst + is[i] * elem_bytes,
                   (const char *)vs + i * elem_bytes, (size_t)elem_bytes);
    }
    return 0;
}

/* Gather: dst[i] := src[is[i]] (array indexing x[i], Section 2.1).  Every
 * index must lie in [0, n_src): returns -1 before writing anything otherwise. */
int ixo_gather(void *dst, const void *src, int64_t n_src, const int64_t *is,
               int64_t m, int64_t elem_bytes) {
    if (n_src < 0 || m < 0 || elem_bytes <= 0) return -1;
    for (int64_t i = 0; i < m; i++)
        if (is[i] < 0 || is[i] >= n_src) return -1;
    for (int64_t i = 0; i < m; i++)
        memcpy((char *)dst + i * elem_bytes,
               (const char *)src + is[i] * elem_bytes, (size_t)elem_bytes);
    return 0;
}

/* Reduce-by-index with min (Futhark's `hist i64.min`, used by
 * get_smallest_pairs in Sections 5.4 and 6 and, for the dynamic verification of
 * scatter, in the evaluation of Section 6).  Every location starts at
 * `neutral`; then each i whose index is[i] lies in [0, n_dst) lowers
 * dst[is[i]] to vs[i] when vs[i] is smaller.  vs == NULL means vs[i] = i. */
int ixo_hist_min(int64_t *dst, int64_t n_dst, int64_t neutral, const int64_t *is,
                 const int64_t *vs, int64_t m) {
    if (n_dst < 0 || m < 0 || (n_dst > 0 && !dst) || (m > 0 && !is)) return -1;
    for (int64_t v = 0; v < n_dst; v++) dst[v] = neutral;
    for (int64_t i = 0; i < m; i++) {
        if (0 <= is[i] && is[i] < n_dst) {
            int64_t x = vs ? vs[i] : i;
            if (x < dst[is[i]]) dst[is[i]] = x;
        }
    }
    return 0;
}

/* get_smallest_pairs (Sections 5.4 and 6, maximal matching): given edge
 * endpoints es (Range es [0, n_verts) is a precondition) and injective edge
 * ids `is`, keep the entries whose id is the least id at their endpoint.  A
 * reduce-by-index with min (neutral n_es) of the ids over the endpoints gives
 * one minimum per vertex; entry k is kept when the minimum at es[k] is is[k];
 * the kept endpoints and ids are then filtered out, in input order.  Entries with es[k] outside [0, n_verts) are not kept (reading: the
 * precondition makes them absent; here they are dropped).  Writes es', is'
 * (capacity m each) and their length to *count. */
int ixo_get_smallest_pairs(int64_t n_verts, int64_t n_es, const int64_t *es, const int64_t *is,
                           int64_t m, int64_t *es_out, int64_t *is_out, int64_t *count) {
    if (n_verts < 0 || m < 0 || !count || (m > 0 && (!es || !is || !es_out || !is_out))) return -1;
    int64_t *H = (int64_t *)malloc((size_t)(n_verts > 0 ? n_verts : 1) * sizeof(int64_t));
    if (!H) return -2;
    ixo_hist_min(H, n_verts, n_es, es, is, m);
    int64_t c = 0;
    for (int64_t k = 0; k < m; k++) {
        int keep = 0 <= es[k] && es[k] < n_verts && H[es[k]] == is[k];
        if (keep) {
            es_out[c] = es[k];
            is_out[c] = is[k];
            c++;
        }
    }
    *count = c;
    free(H);
    return 0;
}

/* Dynamically verified scatter: the "Base" variant of the scatter in
 * partition2 in the evaluation of Section 6 (table "tab:eval", right),
 * which checks at run time that no location is written twice, with a
 * reduce-by-index of atomic minima.  The output starts zeroed; a
 * reduce-by-index with min over the write positions i records, for every
 * location, the least i that writes it (its winner).  Write i is safe when
 * is[i] is out of bounds or i is the winner of is[i].  The verdict holds when
 * every write is safe; otherwise first_violation is the least unsafe i (the
 * earliest second write to a location) and aux = is[i].  Every written
 * location then takes its winner's value, so with injective indices the
 * result is the plain scatter into a zeroed array. */
int ixo_scatter_checked(void *dst, int64_t n_dst, const int64_t *is, const void *vs,
                        int64_t m, int64_t elem_bytes, int64_t *verdict) {
    if (n_dst < 0 || m < 0 || elem_bytes <= 0 || !verdict) return -1;
    if (m > 0 && (!is || !vs)) return -1;
    memset(dst, 0, (size_t)(n_dst * elem_bytes));
    int64_t *win = (int64_t *)malloc((size_t)(n_dst > 0 ? n_dst : 1) * sizeof(int64_t));
    if (!win) return -2;
    ixo_hist_min(win, n_dst, m, is, NULL, m);
    verdict[0] = 1;
    verdict[1] = -1;
    verdict[2] = 0;
    for (int64_t i = 0; i < m; i++) {
        if (0 <= is[i] && is[i] < n_dst && win[is[i]] != i) {
            verdict[0] = 0;
            verdict[1] = i;
            verdict[2] = is[i];
            break;
        }
    }
    for (int64_t v = 0; v < n_dst; v++)
        if (win[v] < m)
            memcpy((char *)dst + v * elem_bytes, (const char *)vs + win[v] * elem_bytes,
                   (size_t)elem_bytes);
    free(win);
    return 0;
}

/* v-way partition (FiltPart with v pairwise exclusive predicates p_1..p_v,
 * Section 2.3, figure "Array Properties": with no filtering, the elements
 * satisfying p_1 come first, then those satisfying p_2, and so on, each class
 * in input order; partition3 of the evaluation, Section 6, is v = 3).
 * The class of element i is the h - 1 of its predicate p_h; the last class is
 * everything no earlier predicate takes (p_v = not (p_1 or ... or p_{v-1})).
 * Class kinds:
 *   IXO_CLASS_MOD:    int32 keys, class = floor-mod(key, v);
 *   IXO_CLASS_THRESH: f32 keys, p_1 = x < s[0], p_h = s[h-2] <= x < s[h-1],
 *                     with s non-decreasing; NaN takes no p_h, h < v, so it
 *                     is in the last class;
 *   IXO_CLASS_BYTES:  class = min(cls[i], v - 1) from a byte array.
 * Steps: the classes; N_c = number of elements of class c; base_c = N_0 +
 * ... + N_{c-1}; idx[i] = base_{c(i)} + (number of earlier elements of
 * class c(i)); ys = scatter zeros idx xs; counts[c] = N_c. */
enum { IXO_CLASS_MOD = 0, IXO_CLASS_THRESH = 1, IXO_CLASS_BYTES = 2 };

static int class_of(int32_t kind, int32_t v, const float *s, const void *xs, const uint8_t *cls,
                    int64_t i) {
    if (kind == IXO_CLASS_MOD) {
        int64_t x = ((const int32_t *)xs)[i];
        int64_t r = x % v;
        return (int)(r < 0 ? r + v : r);
    }
    if (kind == IXO_CLASS_THRESH) {
        float x = ((const float *)xs)[i];
        for (int h = 0; h < v - 1; h++) {
            int lower_ok = h == 0 ? 1 : (s[h - 1] <= x);
            if (lower_ok && x < s[h]) return h;
        }
        return v - 1;
    }
    return cls[i] < v - 1 ? cls[i] : v - 1;
}

int ixo_partition_v(const void *xs, int64_t n, int32_t kind, int32_t v, const float *s,
                    const uint8_t *cls, void *ys, int64_t *idx, int64_t *counts) {
    if (n < 0 || v < 2 || v > 4 || !counts || (n > 0 && (!ys || !idx))) return -1;
    if (kind == IXO_CLASS_BYTES ? (n > 0 && !cls) : (n > 0 && !xs)) return -1;
    if (kind == IXO_CLASS_THRESH)
        for (int h = 1; h < v - 1; h++)
            if (!(s[h - 1] <= s[h])) return -1;
    int *c = (int *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    if (!c) return -2;
    for (int h = 0; h < v; h++) counts[h] = 0;
    for (int64_t i = 0; i < n; i++) {
        c[i] = class_of(kind, v, s, xs, cls, i);
        counts[c[i]]++;
    }
    int64_t base[4], seen[4] = {0, 0, 0, 0};
    base[0] = 0;
    for (int h = 1; h < v; h++) base[h] = base[h - 1] + counts[h - 1];
    for (int64_t i = 0; i < n; i++) idx[i] = base[c[i]] + seen[c[i]]++;
    memset(ys, 0, (size_t)(n * 4));
    ixo_scatter(ys, n, idx, xs ? xs : (const void *)ys, xs ? n : 0, 4);
    free(c);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* partition2 (Section 2.1) by its definition: the elements whose flag is   */
/* set, in input order, followed by the others, in input order.  `indices`  */
/* gives every element its place in that output -- the scatter array whose  */
/* InvFiltPart property the paper proves (Section 2.3).  With T the number  */
/* of set flags, one walk over the input hands out positions 0, 1, ... to    */
/* the trues and T, T+1, ... to the falses; the elements are then scattered */
/* into a zeroed array of length n.                                          */
/*                                                                          */
/* FILTER mode is the paper's `filter` (FiltPart with p^f = p and no        */
/* partitioning predicate): only the trues are kept, in input order, so a   */
/* true gets the number of trues before it and a false gets -1, which the   */
/* scatter into the length-T target ignores.                                */
/* ------------------------------------------------------------------------ */
static int partition2_from_cs(const void *xs, int64_t kb, int64_t n,
                              const uint8_t *cs, int mode, void *ys,
                              int64_t *indices_out, int64_t *num_true_out) {
    size_t nb = (size_t)(n > 0 ? n : 1) * sizeof(int64_t);
    int64_t *indices = indices_out ? indices_out : malloc(nb);
    if (!indices) return -2;

    int64_t num_true = 0;
    for (int64_t i = 0; i < n; i++)
        if (cs[i]) num_true++;

    int64_t next_true = 0, next_false = num_true;
    for (int64_t i = 0; i < n; i++) {
        if (cs[i])
            indices[i] = next_true++;
        else
            indices[i] = mode == IXO_MODE_PARTITION ? next_false++ : -1;
    }
    if (ys) {
        int64_t len = mode == IXO_MODE_PARTITION ? n : num_true;
        memset(ys, 0, (size_t)(len * kb));
        ixo_scatter(ys, len, indices, xs, n, kb);
    }
    if (num_true_out) *num_true_out = num_true;
    if (indices != indices_out) free(indices);
    return 0;
}

int ixo_partition2(const void *xs, int key_t, int64_t n, int pred_kind,
                   int64_t d, int64_t r, float s, const uint8_t *flags_in,
                   int mode, void *ys, int64_t *indices, int64_t *num_true) {
    if (n < 0 || !valid_key_t(key_t)) return -1;
    if (mode != IXO_MODE_PARTITION && mode != IXO_MODE_FILTER) return -1;
    uint8_t *cs = malloc((size_t)(n > 0 ? n : 1));
    if (!cs) return -2;
    int rc = ixo_map_pred(xs, key_t, n, pred_kind, d, r, s, flags_in, cs);
    if (rc == 0)
        rc = partition2_from_cs(xs, key_bytes(key_t), n, cs, mode, ys,
                                indices, num_true);
    free(cs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Segmented helpers (Section 2.1, figure "Running Examples", right).       */
/* ------------------------------------------------------------------------ */

/* sgmSum flags xs (Section 2.1): the running sum of xs that restarts at
 * every set flag, i.e. out[i] = xs[j] + ... + xs[i] with j the last position
 * <= i whose flag is set (j = 0 if there is none).  It is the inclusive scan
 * of (flag, value) pairs under (fx, vx) (+) (fy, vy) = (fx || fy,
 * fy ? vy : vx + vy) with neutral element (false, 0), the reading taken for
 * the operator. */
int ixo_sgm_sum(const uint8_t *flags, const int64_t *xs, int64_t n,
                int64_t *out) {
    if (n < 0) return -1;
    int64_t run = 0;
    for (int64_t i = 0; i < n; i++) {
        run = flags[i] ? xs[i] : run + xs[i];
        out[i] = run;
    }
    return 0;
}

/* mkSgmDescr shape xs (Section 2.1): an array of length sum(shape), zero
 * except at the first position of every non-empty row k, which holds xs[k].
 * Row k starts at o_k, the sum of the sizes of rows 0..k-1; an empty row has
 * no first position and leaves no trace.  `out` must hold sum(shape)
 * entries; returns -1 if a size is negative or the length differs. */
int ixo_mk_sgm_descr(const int64_t *shape, int64_t m, const int64_t *xs,
                     int64_t *out, int64_t out_len) {
    if (m < 0) return -1;
    int64_t len = 0;
    for (int64_t k = 0; k < m; k++) {
        if (shape[k] < 0) return -1;
        len += shape[k];
    }
    if (len != out_len) return -1;
    for (int64_t j = 0; j < len; j++) out[j] = 0;
    int64_t o = 0;
    for (int64_t k = 0; k < m; k++) {
        if (shape[k] > 0) out[o] = xs[k];
        o += shape[k];
    }
    return 0;
}

/* mkII shape (Section 2.1): the row number of every flat element, i.e.
 * out[i] = k for o_k <= i < o_k + shape[k].  The paper's example maps the
 * shape [0,2,1,0,3] to [1,1,2,4,4,4]. */
int ixo_mk_ii(const int64_t *shape, int64_t m, int64_t *out, int64_t out_len) {
    if (m < 0) return -1;
    int64_t len = 0;
    for (int64_t k = 0; k < m; k++) {
        if (shape[k] < 0) return -1;
        len += shape[k];
    }
    if (len != out_len) return -1;
    int64_t i = 0;
    for (int64_t k = 0; k < m; k++)
        for (int64_t j = 0; j < shape[k]; j++) out[i++] = k;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* partition2L -- partition2 applied to every row of a jagged array given by */
/* its shape (Section 6, "Segmented operations").  Row k occupies the flat  */
/* interval [o_k, o_k + shape[k]) with o_k = sum of the earlier sizes; rows  */
/* may be empty.  Each row is partitioned on its own, and its scatter        */
/* indices are shifted by the row offset, so trues of row k land at          */
/* o_k + (#trues before i in the row) and falses at o_k + T_k + (#falses     */
/* before i in the row), T_k = number of trues in row k.  In FILTER mode the */
/* kept elements of row k are packed at o'_k = sum of the earlier rows'      */
/* kept counts (filter_seg) and dropped elements get index -1.               */
/* The descriptor flag array is mkSgmDescr shape (replicate m 1), written as */
/* bytes (1 at the start of every non-empty row, 0 elsewhere).              */
/* ------------------------------------------------------------------------ */
int ixo_partition2L(const void *xs, int key_t, int64_t n, const int64_t *shape,
                    int64_t m, int pred_kind, int64_t d, int64_t r, float s,
                    const uint8_t *flags_in, int mode, void *ys,
                    int64_t *indices, int64_t *seg_split, uint8_t *flags_out) {
    if (n < 0 || m < 0 || !valid_key_t(key_t)) return -1;
    if (mode != IXO_MODE_PARTITION && mode != IXO_MODE_FILTER) return -1;
    int64_t total = 0;
    for (int64_t k = 0; k < m; k++) {
        if (shape[k] < 0) return -1;
        total += shape[k];
    }
    if (total != n) return -1;
    int64_t kb = key_bytes(key_t);
    uint8_t *cs = malloc((size_t)(n > 0 ? n : 1));
    if (!cs) return -2;
    int rc = ixo_map_pred(xs, key_t, n, pred_kind, d, r, s, flags_in, cs);
    if (rc != 0) { free(cs); return rc; }

    int64_t o = 0, okept = 0;
    for (int64_t k = 0; k < m && rc == 0; k++) {
        int64_t sk = shape[k];
        int64_t tk = 0;
        int64_t *loc = malloc((size_t)(sk > 0 ? sk : 1) * sizeof(int64_t));
        if (!loc) { rc = -2; break; }
        rc = partition2_from_cs((const char *)xs + o * kb, kb, sk, cs + o, mode,
                                NULL, loc, &tk);
        if (rc == 0) {
            int64_t base = mode == IXO_MODE_PARTITION ? o : okept;
            for (int64_t i = 0; i < sk; i++) {
                int64_t g = loc[i] < 0 ? -1 : base + loc[i];
                if (indices) indices[o + i] = g;
            }
            if (ys) {
                /* scatter the row into its slice of the output */
                int64_t len = mode == IXO_MODE_PARTITION ? sk : tk;
                char *dst = (char *)ys + base * kb;
                memset(dst, 0, (size_t)(len * kb));
                ixo_scatter(dst, len, loc, (const char *)xs + o * kb, sk, kb);
            }
            if (seg_split) seg_split[k] = tk;
        }
        free(loc);
        o += sk;
        okept += tk;
    }
    if (rc == 0 && flags_out) {
        int64_t *ones = malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
        int64_t *descr = malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
        if (!ones || !descr) rc = -2;
        else {
            for (int64_t k = 0; k < m; k++) ones[k] = 1;
            rc = ixo_mk_sgm_descr(shape, m, ones, descr, n);
            for (int64_t j = 0; rc == 0 && j < n; j++)
                flags_out[j] = (uint8_t)descr[j];
        }
        free(ones); free(descr);
    }
    free(cs);
    return rc;
}

/* partition2L with predicates that depend on the segment number (Section 1:
 * segmented two-way partitioning filters or partitions each row of the jagged
 * array by a predicate of the row number k):
 *   IXO_ROW_LT:  f32 keys, p_k(x) = x < s_rows[k];
 *   IXO_ROW_MOD: int32 keys, p_k(x) = floor-mod(x, d) == floor-mod(k, d).
 * The flags cs are computed row by row, then partition2L runs on them. */
enum { IXO_ROW_LT = 0, IXO_ROW_MOD = 1 };

int ixo_partition2L_rows(const void *xs, int key_t, int64_t n, const int64_t *shape,
                         int64_t m, int row_kind, int64_t d, const float *s_rows, int mode,
                         void *ys, int64_t *indices, int64_t *seg_split, uint8_t *flags_out) {
    if (n < 0 || m < 0 || (n > 0 && !xs)) return -1;
    if (row_kind == IXO_ROW_LT ? (key_t != IXO_F32 || (m > 0 && !s_rows))
                               : (row_kind != IXO_ROW_MOD || key_t != IXO_I32 || d < 1))
        return -1;
    int64_t total = 0;
    for (int64_t k = 0; k < m; k++) {
        if (shape[k] < 0) return -1;
        total += shape[k];
    }
    if (total != n) return -1;
    uint8_t *cs = malloc((size_t)(n > 0 ? n : 1));
    if (!cs) return -2;
    int rc = 0;
    int64_t o = 0;
    int64_t kb = key_bytes(key_t);
    for (int64_t k = 0; k < m && rc == 0; k++) {
        const void *row = (const char *)xs + o * kb;
        if (row_kind == IXO_ROW_LT)
            rc = ixo_map_pred(row, key_t, shape[k], IXO_PRED_LT, 1, 0, s_rows[k], NULL, cs + o);
        else
            rc = ixo_map_pred(row, key_t, shape[k], IXO_PRED_MOD_EQ, d, floor_mod(k, d), 0.f, NULL,
                              cs + o);
        o += shape[k];
    }
    if (rc == 0)
        rc = ixo_partition2L(xs, key_t, n, shape, m, IXO_PRED_FLAGS, 1, 0, 0.f, cs, mode, ys,
                             indices, seg_split, flags_out);
    free(cs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Property checkers (Section 2.3, figure "Array Properties").              */
/* Each writes a verdict {holds, first_violation, aux} as three int64:       */
/* holds is 1 or 0; first_violation is -1 when the property holds.  The      */
/* paper proves properties and never locates a failure, so the index         */
/* conventions below are this library's definitions:                         */
/*   Range [lo,hi): min i with X[i] outside [lo,hi); aux = X[i].             */
/*     (The figure's interval is closed, every use in the paper is           */
/*      half-open; half-open is taken, with explicit bounds.)                */
/*   Monotonic op: min i >= 1 with !(X[i-1] op X[i]) (the later element);    */
/*     aux = 0.  (A bound of j < n-1 would leave the last element            */
/*     unconstrained; j < n is taken.  For a transitive op all-pairs and     */
/*     adjacent pairs agree.)                                                */
/*   Inj Rcd=[lo,hi): min i such that some j < i has X[j] = X[i] in Rcd      */
/*     (the earliest second occurrence); aux = X[i].  Entries outside Rcd    */
/*     are ignored.                                                          */
/*   Bij Rcd=[lo,hi) Img=[ilo,ihi): Inj Rcd, every in-Rcd value lies in Img, */
/*     and the number of in-Rcd entries equals |Img|.  first_violation = min */
/*     of the Inj violation and the first in-Rcd value outside Img (aux =    */
/*     that value); failing only on the count gives first_violation = n and  */
/*     aux = the smallest value of Img that is not attained.                 */
/* ------------------------------------------------------------------------ */
static void verdict_set(int64_t *v, int holds, int64_t fv, int64_t aux) {
    v[0] = holds;
    v[1] = fv;
    v[2] = aux;
}

int ixo_check_range(const int64_t *X, int64_t n, int64_t lo, int64_t hi,
                    int64_t *v) {
    if (n < 0) return -1;
    for (int64_t i = 0; i < n; i++) {
        if (!(lo <= X[i] && X[i] < hi)) {
            verdict_set(v, 0, i, X[i]);
            return 0;
        }
    }
    verdict_set(v, 1, -1, 0);
    return 0;
}

static int mono_ok(int64_t a, int64_t b, int op) {
    switch (op) {
    case IXO_MONO_LE: return a <= b;
    case IXO_MONO_LT: return a < b;
    case IXO_MONO_GE: return a >= b;
    default: return a > b;
    }
}

int ixo_check_mono(const int64_t *X, int64_t n, int op, int64_t *v) {
    if (n < 0 || op < 0 || op > 3) return -1;
    for (int64_t i = 1; i < n; i++) {
        if (!mono_ok(X[i - 1], X[i], op)) {
            verdict_set(v, 0, i, 0);
            return 0;
        }
    }
    verdict_set(v, 1, -1, 0);
    return 0;
}

/* Seen-set over the restricted co-domain [lo,hi): one bit per value. */
typedef struct {
    uint8_t *bits;
    int64_t lo;
} seen_set;

static int seen_init(seen_set *s, int64_t lo, int64_t hi) {
    uint64_t width = (uint64_t)(hi - lo);
    s->lo = lo;
    s->bits = calloc((size_t)(width / 8 + 1), 1);
    return s->bits ? 0 : -2;
}
static int seen_test_and_set(seen_set *s, int64_t x) {
    uint64_t o = (uint64_t)(x - s->lo);
    int was = (s->bits[o >> 3] >> (o & 7)) & 1;
    s->bits[o >> 3] |= (uint8_t)(1u << (o & 7));
    return was;
}
static int seen_test(const seen_set *s, int64_t x) {
    uint64_t o = (uint64_t)(x - s->lo);
    return (s->bits[o >> 3] >> (o & 7)) & 1;
}

/* The bitmap holds hi-lo bits; co-domains wider than 2^40 values are refused. */
static int rcd_ok(int64_t lo, int64_t hi) {
    return lo <= hi && (uint64_t)(hi - lo) <= ((uint64_t)1 << 40);
}

int ixo_check_inj(const int64_t *X, int64_t n, int64_t lo, int64_t hi,
                  int64_t *v) {
    if (n < 0 || !rcd_ok(lo, hi)) return -1;
    seen_set s;
    if (seen_init(&s, lo, hi)) return -2;
    verdict_set(v, 1, -1, 0);
    for (int64_t i = 0; i < n; i++) {
        int64_t x = X[i];
        if (lo <= x && x < hi && seen_test_and_set(&s, x)) {
            verdict_set(v, 0, i, x);
            break;
        }
    }
    free(s.bits);
    return 0;
}

int ixo_check_bij(const int64_t *X, int64_t n, int64_t lo, int64_t hi,
                  int64_t ilo, int64_t ihi, int64_t *v) {
    if (n < 0 || !rcd_ok(lo, hi) || ilo > ihi || ilo < lo || ihi > hi)
        return -1;
    seen_set s;
    if (seen_init(&s, lo, hi)) return -2;
    int64_t count = 0;
    verdict_set(v, 1, -1, 0);
    for (int64_t i = 0; i < n; i++) {
        int64_t x = X[i];
        if (!(lo <= x && x < hi)) continue;
        count++;
        if (seen_test_and_set(&s, x) || !(ilo <= x && x < ihi)) {
            verdict_set(v, 0, i, x);
            break;
        }
    }
    if (v[0] == 1 && count != ihi - ilo) {
        /* Injective and inside Img, yet fewer values than |Img|. */
        int64_t miss = ilo;
        while (miss < ihi && seen_test(&s, miss)) miss++;
        verdict_set(v, 0, n, miss);
    }
    free(s.bits);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* FiltPart check on the outputs of a flat partition (Section 2.3: FiltPart */
/* and InvFiltPart; partition2's postcondition, Section 2.1).                */
/* Inputs: X (the partitioned keys), the predicate, Y (the output keys, n    */
/* entries; in FILTER mode only the first split are compared), Z             */
/* (the scatter indices) and split.  Sub-checks, numbered as the bits of     */
/* aux:                                                                      */
/*   bit 0  Equiv: split == number of elements satisfying p^f-and-p^p        */
/*          (PARTITION: the trues of p; FILTER: the kept elements);          */
/*   bit 1  Bij: PARTITION -- Z restricted to [0,n) is a bijection onto      */
/*          [0,n) (every Z[i] in [0,n), no repeats); FILTER -- kept Z[i] lie */
/*          in [0,split) without repeats, dropped Z[i] lie outside [0,split);*/
/*   bit 2  class order: PARTITION -- Z[i] < split exactly when p holds;     */
/*   bit 3  stability: inside each class Z is strictly increasing in i       */
/*          (InvFiltPart, item (3));                                         */
/*   bit 4  values: Y[Z[i]] == X[i] bit for bit, for every i whose Z[i] is a */
/*          valid position of Y.                                             */
/* holds iff no bit is set; first_violation = the least index i at which an  */
/* index-wise sub-check (bits 1-4) fails, n if only bit 0 fails, -1 if all   */
/* hold.  aux = the set of failing bits over the whole array.                */
/* ------------------------------------------------------------------------ */
int ixo_check_filtpart(const void *X, int key_t, int64_t n, int pred_kind,
                       int64_t d, int64_t r, float s, const uint8_t *flags_in,
                       int mode, const void *Y, const int64_t *Z, int64_t split,
                       int64_t *v) {
    if (n < 0 || !valid_key_t(key_t)) return -1;
    if (mode != IXO_MODE_PARTITION && mode != IXO_MODE_FILTER) return -1;
    int64_t kb = key_bytes(key_t);
    uint8_t *cs = malloc((size_t)(n > 0 ? n : 1));
    if (!cs) return -2;
    int rc = ixo_map_pred(X, key_t, n, pred_kind, d, r, s, flags_in, cs);
    if (rc) { free(cs); return rc; }

    int64_t ntrue = 0;
    for (int64_t i = 0; i < n; i++) ntrue += cs[i];
    int64_t aux = 0;
    int64_t first = -1;
    if (split != ntrue) aux |= 1;

    int64_t ylen = mode == IXO_MODE_PARTITION ? n : split;
    seen_set seen;
    if (seen_init(&seen, 0, n > 0 ? n : 1)) { free(cs); return -2; }
    int has_last[2] = {0, 0};
    int64_t last[2] = {0, 0};
    for (int64_t i = 0; i < n; i++) {
        int64_t z = Z[i];
        int c = cs[i];
        int64_t bad = 0;
        int kept = mode == IXO_MODE_PARTITION || c;
        if (mode == IXO_MODE_PARTITION) {
            if (!(0 <= z && z < n) || seen_test_and_set(&seen, z)) bad |= 2;
            if ((z < split) != (c != 0)) bad |= 4;
        } else {
            if (c) {
                if (!(0 <= z && z < split) || z >= n ||
                    seen_test_and_set(&seen, z))
                    bad |= 2;
            } else if (0 <= z && z < split) {
                bad |= 2;
            }
        }
        if (kept) {
            int cls = mode == IXO_MODE_PARTITION ? c : 1;
            if (has_last[cls] && !(z > last[cls])) bad |= 8;
            has_last[cls] = 1;
            last[cls] = z;
            if (0 <= z && z < ylen && z < n &&
                memcmp((const char *)Y + z * kb, (const char *)X + i * kb,
                       (size_t)kb) != 0)
                bad |= 16;
        }
        if (bad) {
            if (first < 0) first = i;
            aux |= bad;
        }
    }
    free(seen.bits);
    free(cs);
    if (aux == 0) verdict_set(v, 1, -1, 0);
    else verdict_set(v, 0, first >= 0 ? first : n, aux);
    return 0;
}
