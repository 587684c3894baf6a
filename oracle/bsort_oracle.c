/*
 * CPU oracle for length-bucketed bubble sort of words.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the GPU library never does, and the
 * two share no code.
 *
 * What the paper computes (Alyasseri et al., "Parallelize Bubble Sort
 * Algorithm Using OpenMP"):
 *   - Section II, pre-processing phases 2-3: words are put into sub-arrays by
 *     their number of characters, shorter words before longer ones, and each
 *     sub-array is then bubble-sorted in alphabetic order;
 *   - Section III, approach one, step 4: the order within a sub-array is by
 *     the ASCII code of each letter;
 *   - Section II (abstract and method): the size of each sub-array is the
 *     number of words that have that many characters;
 *   - Section I: bubble sort compares each item with the next one and swaps
 *     them if needed, repeating passes until a pass makes no swap;
 *   - "Bubble sort as parallel": the comparison count is n(n-1)/2;
 *   - "Bubble sort in OpenMP": one sub-array per thread, no dependency
 *     between sub-arrays.
 *
 * Readings taken where the paper is silent:
 *   - bytes compare as unsigned 8-bit values (memcmp order);
 *   - sub-arrays are filled in input order and a swap happens only when the
 *     left word is strictly greater, so equal words keep input order;
 *   - a word's "number of characters" is its byte count;
 *   - a length-0 word is legal and forms sub-array 0.
 */
#define _GNU_SOURCE
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_E_INVALID 1
#define ORACLE_E_TOO_LONG 2
#define ORACLE_E_NO_MEMORY 3

/* One slot of a sub-array: the word's bytes and its original index. */
typedef struct {
    const uint8_t *p;
    int32_t idx;
} slot_t;

/*
 * Sub-array construction (Section II phase 2; Section III approach two uses a
 * count array l[] of words per length).  counts[L] = number of words with L
 * bytes, L = 0..max_len.  starts[L] = sum of counts[L'] for L' < L, so
 * starts[max_len+1] = n.  order lists the word indices sub-array by
 * sub-array, each sub-array in input order.
 */
int oracle_bucketize(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                     int32_t n, int32_t max_len,
                     int32_t *counts, int32_t *starts, int32_t *order)
{
    (void)bytes;
    if (n < 0 || max_len < 0) return ORACLE_E_INVALID;
    if (n > 0 && offsets[0] < 0) return ORACLE_E_INVALID;
    for (int32_t i = 0; i < n; ++i) {
        if (offsets[i + 1] < offsets[i] || offsets[i + 1] > n_bytes) return ORACLE_E_INVALID;
        if (offsets[i + 1] - offsets[i] > max_len) return ORACLE_E_TOO_LONG;
    }
    for (int32_t L = 0; L <= max_len; ++L) counts[L] = 0;
    for (int32_t i = 0; i < n; ++i) counts[offsets[i + 1] - offsets[i]] += 1;
    starts[0] = 0;
    for (int32_t L = 0; L <= max_len; ++L) starts[L + 1] = starts[L] + counts[L];
    int32_t *fill = (int32_t *)calloc((size_t)max_len + 1, sizeof(int32_t));
    if (!fill) return ORACLE_E_NO_MEMORY;
    for (int32_t i = 0; i < n; ++i) {
        int32_t L = (int32_t)(offsets[i + 1] - offsets[i]);
        order[starts[L] + fill[L]] = i;
        fill[L] += 1;
    }
    free(fill);
    return ORACLE_OK;
}

/*
 * Bubble sort of one sub-array of m words, all L bytes long (Section I;
 * Section III approach one step 4).  Pass k moves the largest remaining word
 * to position m-1-k by swapping neighbours whose left word is strictly
 * greater.  With early_exit, passes stop after one that makes no swap (the
 * form described in Section I); without it exactly m(m-1)/2 comparisons are
 * made (the count stated in "Bubble sort as parallel").  Returns the number
 * of comparisons.
 */
static int64_t bubble_sort_subarray(slot_t *s, int32_t m, int32_t L, int early_exit)
{
    int64_t comparisons = 0;
    for (int32_t pass = 0; pass + 1 < m; ++pass) {
        int swapped = 0;
        for (int32_t j = 0; j + 1 < m - pass; ++j) {
            comparisons += 1;
            if (memcmp(s[j].p, s[j + 1].p, (size_t)L) > 0) {
                slot_t t = s[j];
                s[j] = s[j + 1];
                s[j + 1] = t;
                swapped = 1;
            }
        }
        if (early_exit && !swapped) break;
    }
    return comparisons;
}

/*
 * The paper's procedure end to end for one list of words: build the
 * sub-arrays, bubble-sort each, concatenate them shortest first (Section II
 * phases 2-3).  perm[k] is the original index of the k-th word of the
 * result.  counts/starts/order are the sub-array sizes, their exclusive scan
 * and the unsorted sub-array contents (see oracle_bucketize); any of them may
 * be NULL.  n_threads > 1 sorts sub-arrays on that many OpenMP threads, one
 * sub-array per thread at a time, largest first ("Bubble sort in OpenMP").
 * On success *comparisons_out (if not NULL) is the total comparison count.
 */
int oracle_bubble_sort(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                       int32_t n, int32_t max_len, int early_exit, int n_threads,
                       int32_t *perm, int32_t *counts, int32_t *starts, int32_t *order,
                       int64_t *comparisons_out)
{
    if (n < 0 || max_len < 0) return ORACLE_E_INVALID;
    int32_t *c = counts ? counts : (int32_t *)malloc(sizeof(int32_t) * ((size_t)max_len + 1));
    int32_t *st = starts ? starts : (int32_t *)malloc(sizeof(int32_t) * ((size_t)max_len + 2));
    int32_t *ord = order ? order : (int32_t *)malloc(sizeof(int32_t) * ((size_t)n + 1));
    slot_t *slots = (slot_t *)malloc(sizeof(slot_t) * ((size_t)n + 1));
    int rc = ORACLE_OK;
    if (!c || !st || !ord || !slots) { rc = ORACLE_E_NO_MEMORY; goto done; }

    rc = oracle_bucketize(bytes, n_bytes, offsets, n, max_len, c, st, ord);
    if (rc != ORACLE_OK) goto done;

    for (int32_t k = 0; k < n; ++k) {
        int32_t i = ord[k];
        slots[k].p = bytes + offsets[i];
        slots[k].idx = i;
    }

    /* sub-arrays, largest first, for the threaded form */
    int32_t nb = max_len + 1;
    int32_t *by_size = (int32_t *)malloc(sizeof(int32_t) * (size_t)nb);
    if (!by_size) { rc = ORACLE_E_NO_MEMORY; goto done; }
    for (int32_t L = 0; L < nb; ++L) by_size[L] = L;
    for (int32_t a = 1; a < nb; ++a) {           /* insertion sort by size, descending */
        int32_t v = by_size[a], b = a - 1;
        while (b >= 0 && c[by_size[b]] < c[v]) { by_size[b + 1] = by_size[b]; --b; }
        by_size[b + 1] = v;
    }
    int64_t total = 0;
#ifdef _OPENMP
    int nt = n_threads > 1 ? n_threads : 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(+:total)
#endif
    for (int32_t q = 0; q < nb; ++q) {
        int32_t L = by_size[q];
        total += bubble_sort_subarray(slots + st[L], c[L], L, early_exit);
    }
    free(by_size);

    for (int32_t k = 0; k < n; ++k) perm[k] = slots[k].idx;
    if (comparisons_out) *comparisons_out = total;

done:
    if (!counts) free(c);
    if (!starts) free(st);
    if (!order) free(ord);
    free(slots);
    return rc;
}

/*
 * The same procedure over R independent word lists stored back to back:
 * list r holds global words req_start[r] .. req_start[r+1]-1 (offsets are
 * global).  perm[g] for g in list r is a list-local index.  With
 * n_threads > 1, lists are spread over threads.  Returns the first error.
 */
int oracle_bubble_sort_batch(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                             const int64_t *req_start, int32_t R, int32_t max_len,
                             int early_exit, int n_threads, int32_t *perm,
                             int64_t *comparisons_out)
{
    int rc_all = ORACLE_OK;
    int64_t total = 0;
#ifdef _OPENMP
    int nt = n_threads > 1 ? n_threads : 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nt) reduction(+:total)
#endif
    for (int32_t r = 0; r < R; ++r) {
        int64_t a = req_start[r], b = req_start[r + 1];
        int64_t cmp = 0;
        int rc = oracle_bubble_sort(bytes, n_bytes, offsets + a, (int32_t)(b - a), max_len,
                                    early_exit, 1, perm + a, NULL, NULL, NULL, &cmp);
        total += cmp;
        if (rc != ORACLE_OK) {
#ifdef _OPENMP
            #pragma omp critical
#endif
            { if (rc_all == ORACLE_OK) rc_all = rc; }
        }
    }
    if (comparisons_out) *comparisons_out = total;
    return rc_all;
}

/*
 * Definition of the result, written out directly: the permutation that
 * orders words by (length, bytes as unsigned, original index).  A library
 * sort (qsort_r) does the ordering; the key is a total order, so the result
 * is unique and qsort's lack of stability does not matter.
 */
typedef struct {
    const uint8_t *bytes;
    const int64_t *offsets;
} def_ctx;

static int cmp_definition(const void *pa, const void *pb, void *arg)
{
    const def_ctx *c = (const def_ctx *)arg;
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    int64_t la = c->offsets[a + 1] - c->offsets[a], lb = c->offsets[b + 1] - c->offsets[b];
    if (la != lb) return la < lb ? -1 : 1;
    int r = memcmp(c->bytes + c->offsets[a], c->bytes + c->offsets[b], (size_t)la);
    if (r != 0) return r;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int oracle_definition_sort(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                           int32_t n, int32_t *perm)
{
    if (n < 0) return ORACLE_E_INVALID;
    for (int32_t i = 0; i < n; ++i)
        if (offsets[i] < 0 || offsets[i + 1] < offsets[i] || offsets[i + 1] > n_bytes)
            return ORACLE_E_INVALID;
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    def_ctx c = {bytes, offsets};
    qsort_r(perm, (size_t)n, sizeof(int32_t), cmp_definition, &c);
    return ORACLE_OK;
}

/* The definition over back-to-back lists (see oracle_bubble_sort_batch);
 * lists are spread over n_threads threads. */
int oracle_definition_sort_batch(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                                 const int64_t *req_start, int32_t R, int n_threads,
                                 int32_t *perm)
{
    int rc_all = ORACLE_OK;
#ifdef _OPENMP
    int nt = n_threads > 1 ? n_threads : 1;
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int32_t r = 0; r < R; ++r) {
        int64_t a = req_start[r], b = req_start[r + 1];
        int rc = oracle_definition_sort(bytes, n_bytes, offsets + a, (int32_t)(b - a), perm + a);
        if (rc != ORACLE_OK) {
#ifdef _OPENMP
            #pragma omp critical
#endif
            { if (rc_all == ORACLE_OK) rc_all = rc; }
        }
    }
    return rc_all;
}

/*
 * Fixed-width big-endian key of a word of L bytes, the oracle's form of the
 * paper's fixed-width word slot (Section III approach two stores every word
 * of a sub-array in a char array of one width): W = ceil(L/8) unsigned
 * 64-bit lanes; lane w holds bytes 8w..8w+7, the first of them in the most
 * significant position, and bytes past L are zero.  For m words (indices
 * idx[0..m-1], all of length L) lanes[w*m + j] is lane w of word idx[j].
 */
int oracle_pack_keys(const uint8_t *bytes, const int64_t *offsets, const int32_t *idx,
                     int32_t m, int32_t L, uint64_t *lanes)
{
    int32_t W = (L + 7) / 8;
    for (int32_t j = 0; j < m; ++j) {
        int32_t i = idx[j];
        if (offsets[i + 1] - offsets[i] != L) return ORACLE_E_INVALID;
        const uint8_t *p = bytes + offsets[i];
        for (int32_t w = 0; w < W; ++w) {
            uint64_t v = 0;
            for (int32_t k = 0; k < 8; ++k) {
                int32_t pos = 8 * w + k;
                uint64_t byte = pos < L ? (uint64_t)p[pos] : 0u;
                v |= byte << (56 - 8 * k);
            }
            lanes[(int64_t)w * m + j] = v;
        }
    }
    return ORACLE_OK;
}

/*
 * Section II, Table 1 rows 2-3: the whole file bubble-sorted without
 * sub-arrays, by alphabetic order (key 0: bytes compared as unsigned, a
 * word that is a prefix of another sorting first) or by word length
 * (key 1); key 2 compares length, then bytes (the bucketed order, reached
 * without buckets).  Bubble passes over the whole list, swapping only a
 * strictly greater left word, so equal keys keep input order.  Returns the
 * comparison count through *comparisons (n(n-1)/2).
 */
static int whole_cmp(const uint8_t *bytes, const int64_t *offsets, int32_t a, int32_t b, int key)
{
    const int64_t la = offsets[a + 1] - offsets[a], lb = offsets[b + 1] - offsets[b];
    if (key == 1 || key == 2) {
        if (la != lb) return la < lb ? -1 : 1;
        if (key == 1) return 0;
    }
    const int64_t m = la < lb ? la : lb;
    const int r = memcmp(bytes + offsets[a], bytes + offsets[b], (size_t)m);
    if (r != 0) return r;
    return la < lb ? -1 : (la > lb ? 1 : 0);
}

int oracle_bubble_sort_whole(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                             int32_t n, int key, int32_t *perm, int64_t *comparisons)
{
    if (n < 0 || key < 0 || key > 2) return ORACLE_E_INVALID;
    for (int32_t i = 0; i < n; ++i)
        if (offsets[i] < 0 || offsets[i + 1] < offsets[i] || offsets[i + 1] > n_bytes)
            return ORACLE_E_INVALID;
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    int64_t cmp = 0;
    for (int32_t pass = 0; pass + 1 < n; ++pass)
        for (int32_t j = 0; j + 1 < n - pass; ++j) {
            ++cmp;
            if (whole_cmp(bytes, offsets, perm[j], perm[j + 1], key) > 0) {
                const int32_t t = perm[j];
                perm[j] = perm[j + 1];
                perm[j + 1] = t;
            }
        }
    *comparisons = cmp;
    return ORACLE_OK;
}

/*
 * Section II pre-processing phase 1 (Section III approach one step 2): the
 * special characters are removed and the text is split into words.  Reading
 * where the paper only gives examples (quote, comma, full stop, question and
 * exclamation marks): a word is a maximal run of ASCII letters A-Z, a-z, and
 * every other byte separates words and is dropped.
 *
 * One pass over the text: a letter is copied to out; the first letter after a
 * non-letter (or at the start) opens a new word at the current output
 * length.  out holds n_bytes bytes, offsets cap_words + 1 entries.  Returns
 * the word count through *n_words and the letter count through *n_letters;
 * ORACLE_E_INVALID if the words do not fit cap_words.
 */
static int is_ascii_letter(uint8_t c)
{
    return (c >= 'A' && c <= 'Z') || (c >= 'a' && c <= 'z');
}

int oracle_tokenize(const uint8_t *text, int64_t n_bytes, uint8_t *out, int64_t *offsets,
                    int64_t cap_words, int64_t *n_words, int64_t *n_letters)
{
    int64_t nw = 0, nl = 0;
    int in_word = 0;
    for (int64_t i = 0; i < n_bytes; ++i) {
        const uint8_t c = text[i];
        if (is_ascii_letter(c)) {
            if (!in_word) {
                if (nw >= cap_words) return ORACLE_E_INVALID;
                offsets[nw++] = nl;
                in_word = 1;
            }
            out[nl++] = c;
        } else {
            in_word = 0;
        }
    }
    offsets[nw] = nl;
    *n_words = nw;
    *n_letters = nl;
    return ORACLE_OK;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
