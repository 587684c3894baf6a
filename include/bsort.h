/*
 * bsort -- length-bucketed odd-even transposition sort of words on AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The operation (Alyasseri et al., "Parallelize Bubble Sort Algorithm Using
 * OpenMP", Section II pre-processing phases 2-3 and Section III approach one
 * step 4): words are distributed into sub-arrays by their number of
 * characters, shorter words before longer ones, and each sub-array is sorted
 * by the ASCII codes of its words' letters.  The paper sorts each sub-array
 * with bubble sort; this library runs bubble sort's data-parallel form,
 * odd-even transposition sort, on tiles of a sub-array, and joins tiles with
 * a block odd-even merge-split.  The result is exact and unique:
 *
 *   perm[k] = index of the k-th word in increasing (length, bytes, index)
 *             order, bytes compared as unsigned 8-bit values (memcmp order),
 *             ties (equal words) in increasing input index.
 *
 * Conventions for every entry point
 *   - Words are given as one byte buffer with no separators plus int64
 *     offsets: word i is bytes[offsets[i] .. offsets[i+1]-1].  Only
 *     bytes[offsets[0] .. offsets[n]-1] is read, so a caller holding a slice
 *     of a longer byte stream may pass bytes = slice - offsets[0].
 *   - Every array argument named "device" is device memory on the current
 *     HIP device, allocated and owned by the caller; the library never frees
 *     or keeps it beyond the call's stream work.  Arrays named "host" are
 *     host memory read during the call only.
 *   - Calls are asynchronous on the given stream (a hipStream_t passed as
 *     void*; NULL is the null stream) unless stated otherwise: the sorting
 *     calls never wait for the device or read anything back (every launch
 *     size is fixed on the host; the merge-split work of sub-arrays larger
 *     than LDS is found on the device by one launch).  Outputs are valid
 *     once the stream reaches the call's work.
 *   - No entry point allocates device memory except bsort_plan_create.
 *     Scratch space is a caller-allocated workspace of at least
 *     bsort_workspace_bytes(...) bytes, 256-byte aligned.  Calls that run
 *     concurrently must use distinct workspaces.
 *   - Objects the library owns: plans (bsort_plan_create .. destroy, each
 *     with its own streams for the capture), and,
 *     per device, up to four pools of three HIP streams (default priority)
 *     with their fork/join events.  A batch sort that fans its in-LDS stages
 *     out (the default; see bsort_sort_batch_staged) takes the pool of its
 *     caller's stream, creating it on first use, and keeps it until the
 *     process ends.  BSORT_FLAG_SERIAL_STAGES runs everything on the
 *     caller's stream and creates nothing.
 *   - Host-side argument checks return a status synchronously and launch
 *     nothing when they fail.  Faults found on the device (a word longer than
 *     max_len, offsets that decrease or point past n_bytes, request bounds
 *     that decrease) set a status word in the workspace, read back by
 *     bsort_get_device_status; the affected words are left out of the
 *     result, and outputs are then unspecified but stay inside their
 *     arrays.  No entry point aborts or throws.
 *   - n_words == 0 is allowed and does nothing.
 */
#ifndef BSORT_H
#define BSORT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Longest word accepted.  Keys are ceil(L/8) uint64 lanes, so at most 8. */
#define BSORT_MAX_LEN 64

typedef enum {
    BSORT_OK = 0,
    BSORT_E_INVALID = 1,     /* bad argument: null pointer, negative size, bad offsets */
    BSORT_E_TOO_LONG = 2,    /* max_len > BSORT_MAX_LEN, or a word longer than max_len */
    BSORT_E_NO_MEMORY = 3,   /* an allocation failed (plans only) */
    BSORT_E_WORKSPACE = 4,   /* workspace too small or misaligned */
    BSORT_E_HIP = 5,         /* a HIP runtime call failed; see bsort_last_error */
    BSORT_E_CAPACITY = 6     /* batch exceeds the capacity a plan was built for */
} bsort_status;

typedef void *bsort_stream_t;   /* hipStream_t */

/* One list of words (one request). */
typedef struct {
    const uint8_t *bytes;    /* device [n_bytes] concatenated word bytes */
    int64_t n_bytes;         /* size of bytes; every offset must be <= n_bytes */
    const int64_t *offsets;  /* device [n_words+1], non-decreasing, offsets[0] >= 0 */
    int32_t n_words;         /* 0 <= n_words < 2^31 */
    int32_t max_len;         /* bound on word length, 0 <= max_len <= BSORT_MAX_LEN */
} bsort_words;

/* Sub-arrays by length (the paper's count array and sub-arrays). */
typedef struct {
    int32_t *counts;         /* device [max_len+1]: counts[L] = words of length L */
    int32_t *starts;         /* device [max_len+2]: exclusive running sum of counts */
    int32_t *order;          /* device [n_words]: word indices grouped by length,
                                shortest first, input order inside each length */
} bsort_buckets;

/* Launch tuning; NULL or zero fields mean the library default. */
typedef struct {
    int32_t tile_keys;       /* words per odd-even transposition tile for sub-arrays sorted
                                in one tile (and in LDS with BSORT_FLAG_LDS_TILE): a power
                                of two in [128, 4096], clamped to 512 and per key width */
    int32_t merge_threads;   /* not used (kept for compatibility): 0, or a multiple of
                                64 in 64..1024 */
    int32_t flags;           /* BSORT_FLAG_* */
    int32_t hbm_tile_keys;   /* tile size for sub-arrays too large for LDS, merged
                                through HBM: a power of two in [128, 8192].  Default (0):
                                the largest tile whose pair fits LDS (8192 words for
                                keys of up to 4 bytes, 4096 up to 12, 2048 up to 16) and
                                2048 for longer keys; clamped per key width and LDS size */
} bsort_tuning;

/* The plain form: the batched form's kernels launched one sub-array at a
 * time -- per list its bucketize launches, then one host synchronisation to
 * read every sub-array's size, then per (request, length) sub-array one sort
 * launch (routed as the batched form routes it) and one launch per
 * merge-split phase.  Same result; for comparison with the batched form.
 * This form waits for the device inside the call. */
#define BSORT_FLAG_PER_BUCKET_LAUNCH 1
/* Testing only: stop after the tile sorts (no merge-split); perm then holds
 * each tile sorted on its own. */
#define BSORT_FLAG_TILES_ONLY 2
/* Run every sort stage in order on the caller's stream instead of fanning
 * the in-LDS classes out over the library's own streams.  Same result;
 * slower, but each stage then has the GPU to itself (per-stage timing) and
 * no work runs outside the caller's stream. */
#define BSORT_FLAG_SERIAL_STAGES 4
/* Testing only: every wait of the merge-split launch gives up at once, as a
 * bounded wait does when the work it waits for never completes: the launch
 * ends, bsort_get_device_status reports BSORT_E_INVALID ("a wait of the
 * merge-split launch gave up") and perm is unspecified. */
#define BSORT_FLAG_STALL_TEST 8
/* Sub-arrays sorted in LDS use tile_keys (clamped to 512 and per key width)
 * as the size of the tiles they sort before merging.  Without it the tile is
 * 512 words for keys of up to 4 bytes and, for longer keys, tile_keys doubled
 * until at most 16 merge-split phases remain (at most 512).  Same result; a
 * knob for the autotuner. */
#define BSORT_FLAG_LDS_TILE 16

/* Workspace bytes for up to total_words words in up to n_requests lists with
 * words of at most max_len bytes.  Returns 0 for invalid arguments. */
size_t bsort_workspace_bytes(int64_t total_words, int32_t max_len, int32_t n_requests);

/*
 * Distribute words into sub-arrays by length (Section II phase 2; Section III
 * approach two's count array): fills b->counts, b->starts and b->order.
 * Stable: inside a length, order keeps input order.
 */
bsort_status bsort_bucketize(const bsort_words *w, const bsort_buckets *b,
                             void *ws, size_t ws_bytes, bsort_stream_t stream);

/*
 * Sort each sub-array made by bsort_bucketize (same w and b) in byte order
 * and write the final order to perm (device [n_words]): Section II phase 3
 * with bubble sort run as odd-even transposition sort, plus block
 * merge-split for sub-arrays longer than one tile.  b is read only.  Use the
 * workspace the matching bsort_bucketize used: bsort_bucketize and
 * bsort_sort_batch clear the device status word when they start, and this
 * call adds its own faults to it.
 */
bsort_status bsort_sort_buckets(const bsort_words *w, const bsort_buckets *b,
                                int32_t *perm, const bsort_tuning *t,
                                void *ws, size_t ws_bytes, bsort_stream_t stream);

/* R independent lists stored back to back. */
typedef struct {
    const uint8_t *bytes;        /* device [n_bytes] */
    int64_t n_bytes;
    const int64_t *offsets;      /* device [total_words+1], global byte offsets */
    const int64_t *req_start;    /* device [n_requests+1]: list r holds global words
                                    req_start[r] .. req_start[r+1]-1; req_start[0] = 0 */
    const int64_t *h_req_start;  /* host copy of req_start (sizes the launch, no sync) */
    int32_t n_requests;
    int32_t max_len;
} bsort_batch;

/*
 * Sort every list of a batch at once: all sub-arrays of all lists go through
 * one sequence of launches.  perm (device [total_words]): for global position
 * g in list r, perm[g] is the list-local index of the word at list-local
 * sorted position g - req_start[r].
 */
bsort_status bsort_sort_batch(const bsort_batch *b, int32_t *perm, const bsort_tuning *t,
                              void *ws, size_t ws_bytes, bsort_stream_t stream);

/*
 * Stage timing.  A batch sort has these stages: "bucketize" (in a batch sort
 * the scatter by length also packs each word's key lanes in place), "pack"
 * (tile planning), one "tiles_d<D>" tile-sort launch per record
 * width D = 2 .. ceil(max_len/4)+1 (D = ceil(L/4)+1 for words of L bytes),
 * one "lds_d<D>_<C>" launch per in-LDS size class of capacity C words for
 * D = 2 .. min(9, ceil(max_len/4)+1) (sub-arrays sorted whole in LDS; C =
 * 1024, 2048, 4096, 8192 where D*4*C <= 144 KiB, and a largest class of
 * 16320, 12288, 9216 or 7168 words for D = 2, 3, 4, 5), and "merge_split"
 * (sub-arrays larger than LDS: their chunks sorted in LDS, then one launch
 * that runs every merge-split phase of every such sub-array).
 * bsort_stage_count(max_len) is their number and bsort_stage_name(max_len, i)
 * the name of stage i (NULL if out of range).
 *
 * bucketize runs on the caller's stream.  pack needs only bucketize's counts
 * and starts, so it runs beside bucketize's final scatter on a library stream
 * and is joined back before the sort stages (with BSORT_FLAG_SERIAL_STAGES,
 * or in bsort_sort_buckets, it follows on the caller's stream).  Then the
 * tile stages and merge_split run on the caller's stream, in that order
 * (merge_split merges the tiles the tile stages sort).  The in-LDS stages
 * touch sub-arrays of their own; they are queued after the tile stages and
 * run concurrently with them and with merge_split on three library streams
 * (default priority), joined back into the caller's stream before the call's
 * work ends.  With
 * BSORT_FLAG_SERIAL_STAGES every stage runs on the caller's stream in the
 * order tiles, in-LDS classes, merge_split.
 *
 * bsort_sort_batch_staged is bsort_sort_batch that also records the caller's
 * HIP events (hipEvent_t passed as void*): events[2i] just before stage i and
 * events[2i+1] just after it, on the stream that runs stage i, so
 * hipEventElapsedTime(events[2i], events[2i+1]) is stage i's device time
 * (with other stages running beside it).  n_events must be
 * 2 * bsort_stage_count(b->max_len); a NULL entry is not recorded (so a
 * caller can time only the stages it needs: each recorded event is a marker
 * in the stream).  The per-bucket form cannot be staged.
 */
int bsort_stage_count(int32_t max_len);
const char *bsort_stage_name(int32_t max_len, int i);
bsort_status bsort_sort_batch_staged(const bsort_batch *b, int32_t *perm, const bsort_tuning *t,
                                     void *ws, size_t ws_bytes, bsort_stream_t stream,
                                     void *const *events, int n_events);

/*
 * Pre-processing (Section II phase 1, Section III approach one step 2):
 * raw text to words.  The paper removes special characters (quote, comma,
 * full stop, question and exclamation marks, ...) and splits the text into
 * words; here a word is a maximal run of ASCII letters [A-Za-z] and every
 * other byte (space, newline, punctuation, digits, bytes >= 0x80) separates
 * words and is dropped.  Words keep their text order and case.
 *
 *   text         device [n_bytes], any alignment; only these bytes are read
 *   words_out    device [n_bytes]: the words' letters back to back (the
 *                first result[1] bytes are written)
 *   offsets_out  device [cap_words + 1]: word i is
 *                words_out[offsets_out[i] .. offsets_out[i+1]), i < result[0]
 *   cap_words    capacity of offsets_out in words; (n_bytes + 1) / 2 always
 *                suffices (a word is at least one letter and a separator)
 *   result       device int64[4], written by the call's stream work:
 *                [0] number of words, [1] number of letters, [2] longest
 *                word in bytes, [3] BSORT_OK or BSORT_E_CAPACITY when
 *                result[0] > cap_words (then only offsets_out[0 .. cap_words)
 *                are written; the counts and result[2] still cover every word)
 *   ws           at least bsort_tokenize_workspace_bytes(n_bytes) bytes,
 *                256-byte aligned
 *
 * The output feeds bsort_bucketize, bsort_sort_buckets and bsort_sort_batch
 * as is (bytes = words_out, offsets = offsets_out, n_words = result[0],
 * max_len >= result[2]).
 * n_bytes == 0 gives no words (offsets_out[0] = 0).
 */
size_t bsort_tokenize_workspace_bytes(int64_t n_bytes);
bsort_status bsort_tokenize(const uint8_t *text, int64_t n_bytes, uint8_t *words_out,
                            int64_t *offsets_out, int64_t cap_words, int64_t *result, void *ws,
                            size_t ws_bytes, bsort_stream_t stream);

/*
 * Unbucketed ablation (Section II, Table 1 rows 2-3: the whole file sorted
 * by alphabetic order, or by word length, without sub-arrays).  Rewrites
 * every word as a key of one width, so that the sorting calls see a single
 * sub-array per list and run the same odd-even transposition sort and
 * merge-split over the whole list:
 *   BSORT_KEY_BYTES         the word's bytes, zero-padded to width
 *                           (alphabetic order; width >= longest word; a
 *                           word holding a 0x00 byte ties with itself cut
 *                           there, since padding is 0x00 too)
 *   BSORT_KEY_LENGTH        one byte holding the length (width 1)
 *   BSORT_KEY_LENGTH_BYTES  the length byte, then the padded bytes (the
 *                           bucketed sort's order; width >= 1 + longest)
 *
 *   bytes, offsets  the words (device, as for the other calls; words whose
 *                   offsets leave [0, n_bytes] are not read and set status)
 *   out             device [n_words * width]
 *   offsets_out     device [n_words + 1]: i * width
 *   status          device int32: 0, or nonzero if a word did not fit the
 *                   width (or is longer than 255 bytes with a length byte);
 *                   written by the call's stream work
 * Sorting (out, offsets_out) with max_len = width gives, per list, the
 * stable order of those keys.
 */
#define BSORT_KEY_BYTES 0
#define BSORT_KEY_LENGTH 1
#define BSORT_KEY_LENGTH_BYTES 2
bsort_status bsort_fixed_width(const uint8_t *bytes, int64_t n_bytes, const int64_t *offsets,
                               int64_t n_words, int32_t width, int32_t mode, uint8_t *out,
                               int64_t *offsets_out, int32_t *status, bsort_stream_t stream);

/*
 * Data-structure ablation (Section III: approach one holds the words as
 * vectors of strings, approach two as a fixed-width character array per
 * length; Tables 2 and 3 time the same sort on each).  Sorts every
 * sub-array of one list made by bsort_bucketize (same w and b) with one
 * workgroup per sub-array running odd-even transposition sort over the
 * whole sub-array (n phases; no tiles, no merge-split), the words held as
 *   BSORT_LAYOUT_PACKED  big-endian key dwords in LDS (a compare reads LDS)
 *   BSORT_LAYOUT_TEXT    positions only; a compare reads both words'
 *                        bytes from the text through order and offsets
 * and writes the same perm as bsort_sort_buckets.  A sub-array must fit
 * 144 KiB of LDS ((ceil(L/4) + 1) * 4 bytes per word packed, 4 text);
 * status (device int32) is 0, or has bit 1 set if a sub-array did not fit
 * (it is left unsorted) and bit 2 if order or offsets pointed outside the
 * words.  Asynchronous on the stream.
 */
#define BSORT_LAYOUT_PACKED 0
#define BSORT_LAYOUT_TEXT 1
bsort_status bsort_oets_buckets(const bsort_words *w, const bsort_buckets *b, int32_t *perm,
                                int32_t layout, int32_t *status, bsort_stream_t stream);

/*
 * A captured batch: bsort_sort_batch's launches recorded once into a HIP
 * graph for batches within the given capacity, then replayed by
 * bsort_plan_execute with one graph launch (plus one small launch that
 * passes the batch's pointers and sizes).  The plan owns a small device
 * buffer, the graph, and three HIP streams (default priority) with their
 * events that only its capture uses; the workspace still comes from the
 * caller and must hold bsort_plan_workspace_bytes(plan) bytes.
 */
typedef struct bsort_plan bsort_plan;
bsort_status bsort_plan_create(bsort_plan **plan, int64_t cap_words, int32_t cap_requests,
                               int64_t cap_request_words, int32_t max_len,
                               const bsort_tuning *t, bsort_stream_t stream);
size_t bsort_plan_workspace_bytes(const bsort_plan *plan);
bsort_status bsort_plan_execute(bsort_plan *plan, const bsort_batch *b, int32_t *perm,
                                void *ws, size_t ws_bytes, bsort_stream_t stream);
void bsort_plan_destroy(bsort_plan *plan);

/*
 * bsort_sort_batch for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * workspace is a static device array of BSORT_STATIC_SCRATCH_BYTES (64 MiB)
 * per GPU, which the library holds from its first use on that GPU
 * until the process ends, so the call takes no workspace argument and
 * allocates nothing (no hipMalloc, no library stream: its stages run in
 * order on the caller's stream, as with BSORT_FLAG_SERIAL_STAGES).  The
 * caller passes the batch and perm as for bsort_sort_batch.
 *   status  device uint32 (may be NULL): written by the call's stream work
 *           with the device status word (0: no fault; otherwise the bits
 *           that bsort_get_device_status decodes)
 * Returns BSORT_E_WORKSPACE, launching nothing, when the batch needs more
 * scratch than the array holds (bsort_workspace_bytes(total, max_len, R) >
 * BSORT_STATIC_SCRATCH_BYTES), and BSORT_E_INVALID for the per-bucket
 * form.  Every call on one GPU uses the same array: calls that overlap on a
 * GPU (two streams, two threads) race and must be ordered by the caller.
 */
#define BSORT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
bsort_status bsort_sort_batch_static(const bsort_batch *b, int32_t *perm, const bsort_tuning *t,
                                     uint32_t *status, bsort_stream_t stream);

/* Synchronises the stream and returns the status word a previous call left
 * in ws (BSORT_OK if none), then clears it. */
bsort_status bsort_get_device_status(void *ws, bsort_stream_t stream);

const char *bsort_status_string(bsort_status s);
/* Detail of the last failure on this thread (e.g. the HIP error string). */
const char *bsort_last_error(void);
/* Library version, e.g. "bsort 0.1 gfx950". */
const char *bsort_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BSORT_H */
