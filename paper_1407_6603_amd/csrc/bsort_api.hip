// C ABI of libbsort: argument checks, workspace layout, launch sequences,
// the plain per-bucket form and captured plans.  See include/bsort.h.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bsort.h"
#include "bsort_internal.h"

using namespace bsort;

namespace {

thread_local std::string g_err;

bsort_status fail(bsort_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(BSORT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kDefaultTile = 256;        // single tiles and in-LDS sub-arrays
constexpr int kDefaultHbmTile = 2048;    // sub-arrays merged through HBM

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Workspace layout: a pure function of (total words, lists, max_len), so the
// size a caller asks for and the layout a call uses always agree.
struct Layout {
    size_t status, job, chunk_begin, chunk_list, chunk_hist, len8, key_off, keys, tiles[kNumD],
        tile_count,
        msub, msorted, mcounts, tile_ph, pcnt, pfill, active, pe, po, ps, mhead, counts, starts,
        order, jobs, lbuckets, lb_count, hchunks[kLdsMaxD + 1], hc_count, pmax;
    int64_t chunk_cap, tile_cap, msub_cap, lb_cap;
    int32_t phase_cap, ml1, dmax, wmax;
    size_t bytes;
};

bool make_layout(int64_t total, int32_t R, int32_t max_len, Layout& L) {
    if (total < 0 || R < 0 || max_len < 0 || max_len > BSORT_MAX_LEN) return false;
    memset(&L, 0, sizeof(L));
    L.ml1 = max_len + 1;
    L.dmax = max_len >= 1 ? dwords_for_len(max_len) : 1;
    L.wmax = lanes_for_len(max_len);
    const int64_t tiles_total = (total + kMinTile - 1) / kMinTile;
    L.chunk_cap = (total + kChunk - 1) / kChunk + R;
    L.tile_cap = tiles_total + 4 * (int64_t)R;
    // a sub-array merged through HBM has two tiles of at least kMinTile words
    L.msub_cap = tiles_total / 2 + 1;
    L.phase_cap = (int32_t)std::min<int64_t>(tiles_total + 2, kMaxPhaseCap);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    L.status = take(256);
    L.job = take(sizeof(Job));
    L.chunk_begin = take(sizeof(int64_t) * ((size_t)R + 1));
    L.chunk_list = take(sizeof(int32_t) * (size_t)L.chunk_cap);
    L.chunk_hist = take(sizeof(int32_t) * (size_t)L.chunk_cap * L.ml1);
    L.len8 = take((size_t)total);
    L.key_off = take(sizeof(int64_t) * (size_t)R * L.ml1);
    L.keys = take(sizeof(uint64_t) * (size_t)L.wmax * (size_t)total);
    for (int D = 2; D <= L.dmax && D <= kMaxD; ++D)
        L.tiles[D] = take(sizeof(TileDesc) * (size_t)L.tile_cap);
    L.tile_count = take(sizeof(int32_t) * kNumD);
    L.lb_cap = 4 * (int64_t)R + 1;                    // a width class covers 4 lengths per list
    L.lbuckets = take(sizeof(LBucket) * (size_t)L.lb_cap * (kLdsMaxD + 1) * kLdsClasses);
    L.lb_count = take(sizeof(int32_t) * 3 * kNumD * kLdsClasses);   // count, back, take
    for (int D = 2; D <= L.dmax && D <= kLdsMaxD; ++D)
        L.hchunks[D] = take(sizeof(LBucket) * (size_t)L.tile_cap);
    L.hc_count = take(sizeof(int32_t) * (kLdsMaxD + 1));
    L.pmax = take(sizeof(int32_t));
    L.msub = take(sizeof(MSub) * (size_t)L.msub_cap);
    L.msorted = take(sizeof(MSub) * (size_t)L.msub_cap);
    L.mcounts = take(2 * sizeof(int32_t));
    L.tile_ph = take(sizeof(int32_t) * (size_t)L.tile_cap);
    L.pcnt = take(sizeof(int32_t) * ((size_t)L.phase_cap + 2));
    L.pfill = take(sizeof(int32_t) * ((size_t)L.phase_cap + 2));
    L.active = take(sizeof(int32_t) * ((size_t)L.phase_cap + 2));
    L.pe = take(sizeof(int64_t) * ((size_t)L.msub_cap + 1));
    L.po = take(sizeof(int64_t) * ((size_t)L.msub_cap + 1));
    L.ps = take(sizeof(int64_t) * ((size_t)L.phase_cap + 1));
    L.mhead = take(4 * sizeof(int64_t));
    L.counts = take(sizeof(int32_t) * (size_t)R * L.ml1);
    L.starts = take(sizeof(int32_t) * (size_t)R * (L.ml1 + 1));
    L.order = take(sizeof(int32_t) * (size_t)total);
    L.jobs = take(sizeof(Job) * (size_t)R);
    L.bytes = off;
    return true;
}

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

bsort_status check_tuning(const bsort_tuning* t) {
    if (!t) return BSORT_OK;
    if (t->tile_keys != 0 && (!pow2(t->tile_keys) || t->tile_keys < kMinTile || t->tile_keys > 4096))
        return fail(BSORT_E_INVALID, "tile_keys must be 0 or a power of two in [128, 4096]");
    if (t->hbm_tile_keys != 0 &&
        (!pow2(t->hbm_tile_keys) || t->hbm_tile_keys < kMinTile || t->hbm_tile_keys > 8192))
        return fail(BSORT_E_INVALID, "hbm_tile_keys must be 0 or a power of two in [128, 8192]");
    if (t->merge_threads != 0 &&
        (t->merge_threads < 64 || t->merge_threads > 1024 || t->merge_threads % 64))
        return fail(BSORT_E_INVALID, "merge_threads must be 0 or a multiple of 64 in [64, 1024]");
    if (t->flags & ~(BSORT_FLAG_PER_BUCKET_LAUNCH | BSORT_FLAG_TILES_ONLY |
                     BSORT_FLAG_SERIAL_STAGES | BSORT_FLAG_STALL_TEST | BSORT_FLAG_LDS_TILE))
        return fail(BSORT_E_INVALID, "unknown flag");
    return BSORT_OK;
}

Bounds make_bounds(const Layout& L, int64_t total, int32_t R, int64_t n_max,
                   const bsort_tuning* t) {
    Bounds b;
    memset(&b, 0, sizeof(b));
    b.total = total;
    b.R = R;
    b.ml1 = L.ml1;
    b.chunk_cap = L.chunk_cap;
    b.tile_cap = L.tile_cap;
    b.dmax = L.dmax;
    b.flags = t ? t->flags : 0;
    const int want = (t && t->tile_keys) ? t->tile_keys : kDefaultTile;
    int64_t pb = 0;
    for (int D = 2; D <= kMaxD; ++D) {
        // single tiles and tiles inside in-LDS sub-arrays
        int T = std::min(std::min(want, kWave * kmax_for(D)), kLdsMaxTile);
        b.tile_keys[D] = T;
        // sub-arrays too large for LDS, merged through HBM: chunks of the
        // largest power of two whose pair fits LDS, sorted by an in-LDS class
        // (D <= kLdsMaxD), else register-sized tiles
        const int want_h = (t && t->hbm_tile_keys) ? t->hbm_tile_keys : 0;
        int Th;
        if (D <= kLdsMaxD) {
            Th = hbm_chunk_max(D);
            if (want_h && want_h < Th) Th = want_h;
            b.hbm_class[D] = hbm_chunk_class(D, Th);
        } else {
            Th = std::min(want_h ? want_h : kDefaultHbmTile, kWave * kmax_for(D));
            b.hbm_class[D] = -1;
        }
        b.hbm_tile_keys[D] = Th;
        if (D > L.dmax) continue;
        int cap = 0;                                   // largest in-LDS sub-array for D
        for (int c = 0; c < kLdsClasses; ++c)
            if (lds_fits(D, c)) cap = std::max(cap, lds_cap(c, D));
        if (n_max > std::max(cap, T))                  // some sub-array may take the HBM path
            pb = std::max<int64_t>(pb, (n_max + Th - 1) / Th);
    }
    b.lb_cap = L.lb_cap;
    b.hbm_merge = pb > 1;
    b.pair_lds = pair_merge_lds(L.dmax);
    return b;
}

// Job for the call, pointers into the workspace per the layout.
Job base_job(const Layout& L, char* ws, const Bounds& b) {
    Job j;
    memset(&j, 0, sizeof(j));
    j.ml1 = L.ml1;
    j.max_len = L.ml1 - 1;
    j.flags = b.flags;
    j.status = (uint32_t*)(ws + L.status);
    j.chunk_begin = (int64_t*)(ws + L.chunk_begin);
    j.chunk_list = (int32_t*)(ws + L.chunk_list);
    j.chunk_hist = (int32_t*)(ws + L.chunk_hist);
    j.len8 = (uint8_t*)(ws + L.len8);
    j.chunk_cap = L.chunk_cap;
    j.key_off = (int64_t*)(ws + L.key_off);
    j.keys = (uint64_t*)(ws + L.keys);
    for (int D = 2; D <= kMaxD; ++D) {
        if (D <= L.dmax) {
            j.tiles[D] = (TileDesc*)(ws + L.tiles[D]);
            j.tile_cap[D] = L.tile_cap;
        }
        j.tile_keys[D] = b.tile_keys[D];
        j.hbm_tile_keys[D] = b.hbm_tile_keys[D];
    }
    for (int D = 2; D <= L.dmax && D <= kLdsMaxD; ++D) j.hchunks[D] = (LBucket*)(ws + L.hchunks[D]);
    j.hc_count = (int32_t*)(ws + L.hc_count);
    j.pmax = (int32_t*)(ws + L.pmax);
    j.lbuckets = (LBucket*)(ws + L.lbuckets);
    j.lb_count = (int32_t*)(ws + L.lb_count);
    j.lb_back = j.lb_count + kNumD * kLdsClasses;
    j.lb_take = j.lb_back + kNumD * kLdsClasses;
    j.lb_cap = L.lb_cap;
    j.tile_count = (int32_t*)(ws + L.tile_count);
    j.msub = (MSub*)(ws + L.msub);
    j.msorted = (MSub*)(ws + L.msorted);
    j.msub_cap = L.msub_cap;
    j.mcounts = (int32_t*)(ws + L.mcounts);
    j.tile_ph = (int32_t*)(ws + L.tile_ph);
    j.mtile_cap = L.tile_cap;
    j.pcnt = (int32_t*)(ws + L.pcnt);
    j.pfill = (int32_t*)(ws + L.pfill);
    j.active = (int32_t*)(ws + L.active);
    j.pe = (int64_t*)(ws + L.pe);
    j.po = (int64_t*)(ws + L.po);
    j.ps = (int64_t*)(ws + L.ps);
    j.mhead = (int64_t*)(ws + L.mhead);
    j.phase_cap = L.phase_cap;
    // a wait of the merge launch gives up after 4 s (100 MHz counter)
    j.stall_ticks = (b.flags & BSORT_FLAG_STALL_TEST) ? -1 : 400000000;
    return j;
}

bsort_status check_ws(const Layout& L, void* ws, size_t ws_bytes) {
    if (!ws) return fail(BSORT_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(BSORT_E_WORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < L.bytes)
        return fail(BSORT_E_WORKSPACE, "workspace has " + std::to_string(ws_bytes) +
                                           " bytes, needs " + std::to_string(L.bytes));
    return BSORT_OK;
}

bsort_status check_words(const bsort_words* w) {
    if (!w) return fail(BSORT_E_INVALID, "words is NULL");
    if (w->max_len < 0) return fail(BSORT_E_INVALID, "max_len < 0");
    if (w->max_len > BSORT_MAX_LEN) return fail(BSORT_E_TOO_LONG, "max_len > BSORT_MAX_LEN");
    if (w->n_words < 0 || w->n_bytes < 0) return fail(BSORT_E_INVALID, "negative size");
    if (w->n_words > 0 && !w->offsets) return fail(BSORT_E_INVALID, "offsets is NULL");
    if (w->n_bytes > 0 && !w->bytes) return fail(BSORT_E_INVALID, "bytes is NULL");
    return BSORT_OK;
}

bsort_status check_buckets(const bsort_buckets* b, int32_t n) {
    if (!b || !b->counts || !b->starts) return fail(BSORT_E_INVALID, "buckets arrays are NULL");
    if (n > 0 && !b->order) return fail(BSORT_E_INVALID, "order is NULL");
    return BSORT_OK;
}

// job of a single list (words w) with req_start held inside the device job
Job single_job(const Layout& L, char* ws, Job* jdst, const Bounds& bd, const bsort_words* w) {
    Job j = base_job(L, ws, bd);
    j.bytes = w->bytes;
    j.n_bytes = w->n_bytes;
    j.offsets = w->offsets;
    j.total = w->n_words;
    j.R = 1;
    j.max_len = w->max_len;
    j.rs_inline[0] = 0;
    j.rs_inline[1] = w->n_words;
    j.req_start = (const int64_t*)((char*)jdst + offsetof(Job, rs_inline));
    return j;
}

bsort_status plain_form(const bsort_batch* b, int32_t* perm, const bsort_tuning* t,
                        const Layout& L, char* ws, hipStream_t s);

}  // namespace

struct FanPool;

struct bsort_plan {
    int64_t cap_words;
    int64_t cap_req;
    int32_t cap_R;
    int32_t max_len;
    bsort_tuning tun;
    Layout lay;
    Bounds bd;
    Job* job_dev;
    hipGraphExec_t exec;
    FanPool* fan;            // the plan's own library streams and events (captured into its graph)
};

extern "C" {

size_t bsort_workspace_bytes(int64_t total_words, int32_t max_len, int32_t n_requests) {
    Layout L;
    if (!make_layout(total_words, n_requests, max_len, L)) return 0;
    return L.bytes;
}

bsort_status bsort_fixed_width(const uint8_t* bytes, int64_t n_bytes, const int64_t* offsets,
                               int64_t n_words,
                               int32_t width, int32_t mode, uint8_t* out, int64_t* offsets_out,
                               int32_t* status, bsort_stream_t stream) {
    if (n_words < 0 || n_bytes < 0 || width < 1) return fail(BSORT_E_INVALID, "bad size");
    if (mode != BSORT_KEY_BYTES && mode != BSORT_KEY_LENGTH && mode != BSORT_KEY_LENGTH_BYTES)
        return fail(BSORT_E_INVALID, "unknown key mode");
    if (mode == BSORT_KEY_LENGTH && width != 1)
        return fail(BSORT_E_INVALID, "a length key is one byte wide");
    if (width > BSORT_MAX_LEN) return fail(BSORT_E_TOO_LONG, "width > BSORT_MAX_LEN");
    if (!offsets || !offsets_out || !status) return fail(BSORT_E_INVALID, "NULL pointer");
    if (n_words > 0 && (!bytes || !out)) return fail(BSORT_E_INVALID, "NULL pointer");
    HIP_TRY(launch_fixed_width(bytes, n_bytes, offsets, n_words, width, mode, out, offsets_out,
                               status, (hipStream_t)stream));
    return BSORT_OK;
}

bsort_status bsort_oets_buckets(const bsort_words* w, const bsort_buckets* b, int32_t* perm,
                                int32_t layout, int32_t* status, bsort_stream_t stream) {
    bsort_status st = check_words(w);
    if (st != BSORT_OK) return st;
    if ((st = check_buckets(b, w->n_words)) != BSORT_OK) return st;
    if (layout != BSORT_LAYOUT_PACKED && layout != BSORT_LAYOUT_TEXT)
        return fail(BSORT_E_INVALID, "unknown layout");
    if (!status) return fail(BSORT_E_INVALID, "status is NULL");
    if (w->n_words > 0 && !perm) return fail(BSORT_E_INVALID, "perm is NULL");
    HIP_TRY(launch_layout_oets(w->bytes, w->n_bytes, w->offsets, w->n_words, w->max_len,
                               b->counts, b->starts, b->order, perm, layout, status,
                               (hipStream_t)stream));
    return BSORT_OK;
}

size_t bsort_tokenize_workspace_bytes(int64_t n_bytes) {
    return n_bytes < 0 ? 0 : tok_workspace_bytes(n_bytes);
}

bsort_status bsort_tokenize(const uint8_t* text, int64_t n_bytes, uint8_t* words_out,
                            int64_t* offsets_out, int64_t cap_words, int64_t* result, void* ws,
                            size_t ws_bytes, bsort_stream_t stream) {
    if (n_bytes < 0 || cap_words < 0) return fail(BSORT_E_INVALID, "negative size");
    if (!offsets_out || !result) return fail(BSORT_E_INVALID, "offsets_out or result is NULL");
    if (n_bytes > 0 && (!text || !words_out))
        return fail(BSORT_E_INVALID, "text or words_out is NULL");
    if (n_bytes > ((int64_t)1 << 42)) return fail(BSORT_E_INVALID, "text longer than 4 TiB");
    const size_t need = tok_workspace_bytes(n_bytes);
    if (!ws || ws_bytes < need) return fail(BSORT_E_WORKSPACE, "workspace too small");
    if ((uintptr_t)ws & 255) return fail(BSORT_E_WORKSPACE, "workspace not 256-byte aligned");
    HIP_TRY(launch_tokenize(text, n_bytes, words_out, offsets_out, cap_words, result, ws,
                            (hipStream_t)stream));
    return BSORT_OK;
}

bsort_status bsort_bucketize(const bsort_words* w, const bsort_buckets* b, void* ws,
                             size_t ws_bytes, bsort_stream_t stream) {
    bsort_status st = check_words(w);
    if (st != BSORT_OK) return st;
    if ((st = check_buckets(b, w->n_words)) != BSORT_OK) return st;
    Layout L;
    make_layout(w->n_words, 1, w->max_len, L);
    if ((st = check_ws(L, ws, ws_bytes)) != BSORT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Bounds bd = make_bounds(L, w->n_words, 1, w->n_words, nullptr);
    Job* jd = (Job*)((char*)ws + L.job);
    Job j = single_job(L, (char*)ws, jd, bd, w);
    j.counts = b->counts;
    j.starts = b->starts;
    j.order = b->order;
    HIP_TRY(launch_set_job(j, jd, s));
    HIP_TRY(launch_bucketize(jd, bd, s));
    return BSORT_OK;
}

static hipError_t enqueue_sort(const Job* J, const Bounds& b, hipStream_t s, bool bucketize,
                               void* const* ev, FanPool* own);

bsort_status bsort_sort_buckets(const bsort_words* w, const bsort_buckets* b, int32_t* perm,
                                const bsort_tuning* t, void* ws, size_t ws_bytes,
                                bsort_stream_t stream) {
    bsort_status st = check_words(w);
    if (st != BSORT_OK) return st;
    if ((st = check_buckets(b, w->n_words)) != BSORT_OK) return st;
    if ((st = check_tuning(t)) != BSORT_OK) return st;
    if (w->n_words > 0 && !perm) return fail(BSORT_E_INVALID, "perm is NULL");
    if (t && (t->flags & BSORT_FLAG_PER_BUCKET_LAUNCH))
        return fail(BSORT_E_INVALID, "the per-bucket form is a bsort_sort_batch flag");
    Layout L;
    make_layout(w->n_words, 1, w->max_len, L);
    if ((st = check_ws(L, ws, ws_bytes)) != BSORT_OK) return st;
    if (w->n_words == 0) return BSORT_OK;
    hipStream_t s = (hipStream_t)stream;
    Bounds bd = make_bounds(L, w->n_words, 1, w->n_words, t);
    Job* jd = (Job*)((char*)ws + L.job);
    Job j = single_job(L, (char*)ws, jd, bd, w);
    j.counts = b->counts;
    j.starts = b->starts;
    j.order = b->order;
    j.perm = perm;
    HIP_TRY(launch_set_job(j, jd, s));
    HIP_TRY(enqueue_sort(jd, bd, s, false, nullptr, nullptr));
    return BSORT_OK;
}

static bsort_status check_batch(const bsort_batch* b, int32_t* perm, int64_t& total,
                                int64_t& n_max) {
    if (!b) return fail(BSORT_E_INVALID, "batch is NULL");
    if (b->n_requests < 0) return fail(BSORT_E_INVALID, "n_requests < 0");
    if (b->max_len < 0) return fail(BSORT_E_INVALID, "max_len < 0");
    if (b->max_len > BSORT_MAX_LEN) return fail(BSORT_E_TOO_LONG, "max_len > BSORT_MAX_LEN");
    if (b->n_bytes < 0) return fail(BSORT_E_INVALID, "n_bytes < 0");
    total = 0;
    n_max = 0;
    if (b->n_requests == 0) return BSORT_OK;
    if (!b->h_req_start || !b->req_start) return fail(BSORT_E_INVALID, "req_start is NULL");
    if (b->h_req_start[0] != 0) return fail(BSORT_E_INVALID, "req_start[0] != 0");
    for (int32_t r = 0; r < b->n_requests; ++r) {
        const int64_t n = b->h_req_start[r + 1] - b->h_req_start[r];
        if (n < 0) return fail(BSORT_E_INVALID, "req_start decreases");
        if (n > INT32_MAX) return fail(BSORT_E_INVALID, "a list has 2^31 words or more");
        n_max = std::max(n_max, n);
    }
    total = b->h_req_start[b->n_requests];
    if (total > 0 && (!b->offsets || !perm)) return fail(BSORT_E_INVALID, "offsets or perm NULL");
    if (b->n_bytes > 0 && !b->bytes) return fail(BSORT_E_INVALID, "bytes is NULL");
    return BSORT_OK;
}

static Job batch_job(const Layout& L, char* ws, const Bounds& bd, const bsort_batch* b,
                     int64_t total, int32_t* perm) {
    Job j = base_job(L, ws, bd);
    j.bytes = b->bytes;
    j.n_bytes = b->n_bytes;
    j.offsets = b->offsets;
    j.req_start = b->req_start;
    j.total = total;
    j.R = b->n_requests;
    j.max_len = b->max_len;
    j.counts = (int32_t*)(ws + L.counts);
    j.starts = (int32_t*)(ws + L.starts);
    j.order = (int32_t*)(ws + L.order);
    j.perm = perm;
    if (bd.fused_pack) j.flags |= kJobFusedPack;
    return j;
}

// stages: bucketize, pack, tiles_d2..tiles_d<dmax>, then one stage per in-LDS
// size class, lds_d<D>_<capacity> for D = 2..min(9, dmax), then merge_split
static int stage_dmax(int32_t max_len) { return max_len >= 1 ? dwords_for_len(max_len) : 1; }
static int stage_lds_max(int32_t max_len) { return std::min(stage_dmax(max_len), kLdsMaxD); }

struct StageNames {
    char tiles[kNumD][16];
    char lds[kLdsMaxD + 1][kLdsClasses][24];
    StageNames() {
        for (int D = 0; D < kNumD; ++D) snprintf(tiles[D], sizeof tiles[D], "tiles_d%d", D);
        for (int D = 0; D <= kLdsMaxD; ++D)
            for (int c = 0; c < kLdsClasses; ++c)
                snprintf(lds[D][c], sizeof lds[D][c], "lds_d%d_%d", D, lds_cap(c, D));
    }
};
static const StageNames& stage_names() {
    static const StageNames n;
    return n;
}

// the in-LDS stages in order: (D, class) pairs
static int lds_stages(int32_t max_len, int* Ds, int* cs) {
    int k = 0;
    for (int D = 2; D <= stage_lds_max(max_len); ++D)
        for (int c = 0; c < kLdsClasses; ++c)
            if (lds_fits(D, c)) {
                if (Ds) Ds[k] = D;
                if (cs) cs[k] = c;
                ++k;
            }
    return k;
}

int bsort_stage_count(int32_t max_len) {
    if (max_len < 0 || max_len > BSORT_MAX_LEN) return 0;
    const int nd = stage_dmax(max_len) - 1;
    return 3 + (nd > 0 ? nd : 0) + lds_stages(max_len, nullptr, nullptr);
}

const char* bsort_stage_name(int32_t max_len, int i) {
    const int n = bsort_stage_count(max_len);
    if (i < 0 || i >= n) return nullptr;
    if (i == 0) return "bucketize";
    if (i == 1) return "pack";
    if (i == n - 1) return "merge_split";
    const int nd = stage_dmax(max_len) - 1;
    if (i - 2 < nd) return stage_names().tiles[i];     // i = 2 .. nd+1 -> D = i
    int Ds[(kLdsMaxD + 1) * kLdsClasses], cs[(kLdsMaxD + 1) * kLdsClasses];
    lds_stages(max_len, Ds, cs);
    const int k = i - 2 - nd;
    return stage_names().lds[Ds[k]][cs[k]];
}

// ---- concurrent sort stages
//
// After the key pack the sort stages fall into independent groups: the
// in-LDS size classes each sort sub-arrays of their own, while the
// register-tile sorts must precede the merge-split phases through HBM (those
// merge tiles the tile sorts made).  The tile sorts and the merge-split run
// in order on the caller's stream; the in-LDS classes, largest first, go
// round-robin onto kFan-1 library streams of default priority between a
// fork and a join event, so the last partial round of one stage overlaps the
// others.  Library streams come from a few pools per device, picked by the
// caller's stream; a pool is locked while a call enqueues (its events are
// reused), and graph capture forks and joins the same way.
constexpr int kFan = 4;
constexpr int kFanPools = 4;
constexpr int kMaxDevices = 64;

struct FanPool {
    std::mutex mu;
    bool ready = false;             // streams and fork/join events
    hipStream_t aux[kFan - 1] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kFan - 1] = {};
    hipEvent_t prep_fork = nullptr;  // the plan beside the scatter, on aux[0]
    hipEvent_t prep_join = nullptr;
};

static FanPool g_fan[kMaxDevices][kFanPools];

// caller streams get pools round-robin in order of first use, so a few
// streams working side by side do not queue behind each other
static int fan_pool_for(int dev, hipStream_t s) {
    static std::mutex mu;
    static std::vector<std::pair<hipStream_t, int>> seen[kMaxDevices];
    static int next[kMaxDevices];
    std::lock_guard<std::mutex> lock(mu);
    for (const auto& kv : seen[dev])
        if (kv.first == s) return kv.second;
    const int k = next[dev]++ % kFanPools;
    if (seen[dev].size() < 256) seen[dev].push_back({s, k});
    return k;
}

static hipError_t fan_init(FanPool& f) {
    if (f.ready) return hipSuccess;
    hipError_t e = hipEventCreateWithFlags(&f.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&f.prep_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&f.prep_join, hipEventDisableTiming);
    for (int k = 0; k < kFan - 1 && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&f.aux[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&f.join[k], hipEventDisableTiming);
    }
    if (e == hipSuccess) f.ready = true;
    return e;
}

// a pool's streams and events (a plan's own pool, when the plan is destroyed)
static void fan_destroy(FanPool& f) {
    if (!f.ready) return;
    for (int k = 0; k < kFan - 1; ++k) {
        if (f.aux[k]) (void)hipStreamDestroy(f.aux[k]);
        if (f.join[k]) (void)hipEventDestroy(f.join[k]);
    }
    if (f.fork) (void)hipEventDestroy(f.fork);
    if (f.prep_fork) (void)hipEventDestroy(f.prep_fork);
    if (f.prep_join) (void)hipEventDestroy(f.prep_join);
    f.ready = false;
}

enum StageKind { kStageTiles, kStageLds, kStageMerge };
struct StageRef {
    int kind, D, c, index;   // index: position in bsort_stage_name order
};

// the sort stages after the pack: lane 0 (caller's stream) holds the tile
// sorts then the merge-split; the in-LDS classes follow, largest first
static std::vector<StageRef> sort_stages(const Bounds& b) {
    const int nd = b.dmax - 1;
    std::vector<StageRef> v;
    int Ds[(kLdsMaxD + 1) * kLdsClasses], cs[(kLdsMaxD + 1) * kLdsClasses];
    const int nl = lds_stages(b.ml1 - 1, Ds, cs);
    for (int D = 2; D <= b.dmax && D <= kMaxD; ++D) v.push_back({kStageTiles, D, 0, D});
    v.push_back({kStageMerge, 0, 0, 2 + nd + nl});    // merge_split is the last stage name
    for (int c = kLdsClasses - 1; c >= 0; --c)
        for (int k = 0; k < nl; ++k)
            if (cs[k] == c) v.push_back({kStageLds, Ds[k], c, 2 + nd + k});
    return v;
}

static hipError_t run_stage(const StageRef& st, const Job* J, const Bounds& b, hipStream_t s) {
    switch (st.kind) {
        case kStageTiles: return launch_oets_tiles_one(J, b, st.D, s);
        case kStageLds: return launch_lds_class(J, b, st.D, st.c, s);
        default: return launch_merges(J, b, s);
    }
}

// Everything after the job descriptor: bucketize (if asked), prep and pack,
// then the sort stages fanned out and joined back.  With the library streams
// and a bucketize pass, the plan (which needs only counts and starts) runs on
// a library stream beside the scatter; otherwise everything before the sort
// stages is on the caller's stream.
// ev (optional): 2 events per stage in bsort_stage_name order, recorded just
// before and after the stage on the stream that runs it.  Nothing is read
// back: every launch size is fixed on the host, and the merge-split phases run
// in one launch that finds its work on the device.
// own: the pool to fan out over (a plan's own); else the pool of the caller's stream
static hipError_t enqueue_sort(const Job* J, const Bounds& b, hipStream_t s, bool bucketize,
                               void* const* ev, FanPool* own) {
    auto rec = [&](int i, int end, hipStream_t x) -> hipError_t {
        return ev && ev[2 * i + end] ? hipEventRecord((hipEvent_t)ev[2 * i + end], x) : hipSuccess;
    };
    hipError_t e = hipSuccess;
    // BSORT_FLAG_SERIAL_STAGES: every stage on s and no library stream
    const bool fan = !(b.flags & BSORT_FLAG_SERIAL_STAGES);
    const bool prep_beside = fan && bucketize && b.fused_pack;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    FanPool& f = own ? *own : g_fan[dev][fan ? fan_pool_for(dev, s) : 0];
    std::unique_lock<std::mutex> lock(f.mu, std::defer_lock);
    if (fan) {
        lock.lock();
        if ((e = fan_init(f)) != hipSuccess) return e;
    }
    if (bucketize) {
        if ((e = rec(0, 0, s)) != hipSuccess) return e;
        if ((e = launch_bucket_starts(J, b, s)) != hipSuccess) return e;
        if (prep_beside) {
            hipStream_t x = f.aux[0];
            if ((e = hipEventRecord(f.prep_fork, s)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(x, f.prep_fork, 0)) != hipSuccess) return e;
            if ((e = rec(1, 0, x)) != hipSuccess) return e;
            if ((e = launch_sort_prep(J, b, true, x)) != hipSuccess) return e;
            if ((e = rec(1, 1, x)) != hipSuccess) return e;
            if ((e = hipEventRecord(f.prep_join, x)) != hipSuccess) return e;
        }
        if ((e = launch_scatter(J, b, s)) != hipSuccess) return e;
        if ((e = rec(0, 1, s)) != hipSuccess) return e;
        if (prep_beside && (e = hipStreamWaitEvent(s, f.prep_join, 0)) != hipSuccess) return e;
    }
    if (!prep_beside) {
        if ((e = rec(1, 0, s)) != hipSuccess) return e;
        if ((e = launch_sort_prep(J, b, bucketize, s)) != hipSuccess) return e;
        if ((e = rec(1, 1, s)) != hipSuccess) return e;
    }
    hipStream_t st[kFan] = {s, f.aux[0], f.aux[1], f.aux[2]};
    if (fan) {
        if ((e = hipEventRecord(f.fork, s)) != hipSuccess) return e;
        for (int k = 1; k < kFan; ++k)
            if ((e = hipStreamWaitEvent(st[k], f.fork, 0)) != hipSuccess) return e;
    }
    const std::vector<StageRef> stages = sort_stages(b);
    // the tile sorts first on the caller's stream (short; the merge-split
    // waits on them), then the in-LDS classes round-robin on the library
    // streams, then the merge-split after the tiles on the caller's stream.
    // The classes come in (capacity level, record width) order, so plain
    // round-robin gives each library stream one record width (faster for
    // eager calls).  A plan's capture turns the assignment one stream
    // further at each capacity level, so each stream's chain mixes widths
    // and the chains are of more even length: the runtime replays a graph on
    // streams of its own, which need not keep one chain per queue, and there
    // even chains were measured faster.
    const bool rotate = own != nullptr;
    for (const StageRef& g : stages) {
        if (g.kind != kStageTiles) continue;
        if ((e = rec(g.index, 0, s)) != hipSuccess) return e;
        if ((e = run_stage(g, J, b, s)) != hipSuccess) return e;
        if ((e = rec(g.index, 1, s)) != hipSuccess) return e;
    }
    int lds_seen = 0;
    for (const StageRef& g : stages) {
        if (g.kind != kStageLds) continue;
        const int rr = rotate ? lds_seen + lds_seen / (kFan - 1) : lds_seen;
        ++lds_seen;
        hipStream_t x = fan ? st[1 + rr % (kFan - 1)] : s;
        if ((e = rec(g.index, 0, x)) != hipSuccess) return e;
        if ((e = run_stage(g, J, b, x)) != hipSuccess) return e;
        if ((e = rec(g.index, 1, x)) != hipSuccess) return e;
    }
    for (const StageRef& g : stages) {
        if (g.kind != kStageMerge) continue;
        if ((e = rec(g.index, 0, s)) != hipSuccess) return e;
        if ((e = run_stage(g, J, b, s)) != hipSuccess) return e;
        if ((e = rec(g.index, 1, s)) != hipSuccess) return e;
    }
    for (int k = 1; fan && k < kFan; ++k) {
        if ((e = hipEventRecord(f.join[k - 1], st[k])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, f.join[k - 1], 0)) != hipSuccess) return e;
    }
    return hipGetLastError();
}

static bsort_status sort_batch_impl(const bsort_batch* b, int32_t* perm, const bsort_tuning* t,
                                    void* ws, size_t ws_bytes, bsort_stream_t stream,
                                    void* const* events, int n_events) {
    int64_t total, n_max;
    bsort_status st = check_batch(b, perm, total, n_max);
    if (st != BSORT_OK) return st;
    if ((st = check_tuning(t)) != BSORT_OK) return st;
    if (events) {
        if (n_events != 2 * bsort_stage_count(b->max_len))
            return fail(BSORT_E_INVALID, "n_events must be 2 * bsort_stage_count(max_len)");
        if (t && (t->flags & BSORT_FLAG_PER_BUCKET_LAUNCH))
            return fail(BSORT_E_INVALID, "the per-bucket form cannot be staged");
    }
    Layout L;
    make_layout(total, b->n_requests, b->max_len, L);
    if ((st = check_ws(L, ws, ws_bytes)) != BSORT_OK) return st;
    if (b->n_requests == 0) return BSORT_OK;
    hipStream_t s = (hipStream_t)stream;
    if (t && (t->flags & BSORT_FLAG_PER_BUCKET_LAUNCH))
        return plain_form(b, perm, t, L, (char*)ws, s);
    Bounds bd = make_bounds(L, total, b->n_requests, n_max, t);
    bd.fused_pack = 1;                                 // bucketize runs in this call
    Job* jd = (Job*)((char*)ws + L.job);
    Job j = batch_job(L, (char*)ws, bd, b, total, perm);
    HIP_TRY(launch_set_job(j, jd, s));
    HIP_TRY(enqueue_sort(jd, bd, s, true, events, nullptr));
    return BSORT_OK;
}

bsort_status bsort_sort_batch(const bsort_batch* b, int32_t* perm, const bsort_tuning* t,
                              void* ws, size_t ws_bytes, bsort_stream_t stream) {
    return sort_batch_impl(b, perm, t, ws, ws_bytes, stream, nullptr, 0);
}

bsort_status bsort_sort_batch_staged(const bsort_batch* b, int32_t* perm, const bsort_tuning* t,
                                     void* ws, size_t ws_bytes, bsort_stream_t stream,
                                     void* const* events, int n_events) {
    if (!events) return fail(BSORT_E_INVALID, "events is NULL");
    return sort_batch_impl(b, perm, t, ws, ws_bytes, stream, events, n_events);
}

bsort_status bsort_plan_create(bsort_plan** plan, int64_t cap_words, int32_t cap_requests,
                               int64_t cap_request_words, int32_t max_len,
                               const bsort_tuning* t, bsort_stream_t stream) {
    (void)stream;
    if (!plan) return fail(BSORT_E_INVALID, "plan is NULL");
    *plan = nullptr;
    if (cap_words < 0 || cap_requests < 1 || cap_request_words < 0 || max_len < 0)
        return fail(BSORT_E_INVALID, "bad capacity");
    if (max_len > BSORT_MAX_LEN) return fail(BSORT_E_TOO_LONG, "max_len > BSORT_MAX_LEN");
    bsort_status st = check_tuning(t);
    if (st != BSORT_OK) return st;
    if (t && (t->flags & BSORT_FLAG_PER_BUCKET_LAUNCH))
        return fail(BSORT_E_INVALID, "a plan cannot use the per-bucket form");
    bsort_plan* p = new (std::nothrow) bsort_plan();
    if (!p) return fail(BSORT_E_NO_MEMORY, "plan allocation");
    p->cap_words = cap_words;
    p->cap_req = std::min<int64_t>(cap_request_words, cap_words);
    p->cap_R = cap_requests;
    p->max_len = max_len;
    memset(&p->tun, 0, sizeof(p->tun));
    if (t) p->tun = *t;
    make_layout(cap_words, cap_requests, max_len, p->lay);
    p->bd = make_bounds(p->lay, cap_words, cap_requests, p->cap_req, t);
    p->bd.fused_pack = 1;
    p->job_dev = nullptr;
    p->exec = nullptr;
    // the plan's own library streams and events: a capture never shares
    // streams with eager calls (or with other plans) while it records
    p->fan = new (std::nothrow) FanPool();
    if (!p->fan) {
        delete p;
        return fail(BSORT_E_NO_MEMORY, "plan allocation");
    }
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipError_t e = hipMalloc((void**)&p->job_dev, sizeof(Job));
    if (e != hipSuccess) {
        delete p->fan;
        delete p;
        return fail(BSORT_E_NO_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = fan_init(*p->fan);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t e1 = enqueue_sort(p->job_dev, p->bd, cs, true, nullptr, p->fan);
        e = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        (void)hipFree(p->job_dev);
        fan_destroy(*p->fan);
        delete p->fan;
        delete p;
        return fail(BSORT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *plan = p;
    return BSORT_OK;
}

size_t bsort_plan_workspace_bytes(const bsort_plan* plan) { return plan ? plan->lay.bytes : 0; }

bsort_status bsort_plan_execute(bsort_plan* p, const bsort_batch* b, int32_t* perm, void* ws,
                                size_t ws_bytes, bsort_stream_t stream) {
    if (!p) return fail(BSORT_E_INVALID, "plan is NULL");
    int64_t total, n_max;
    bsort_status st = check_batch(b, perm, total, n_max);
    if (st != BSORT_OK) return st;
    if (b->n_requests > p->cap_R || total > p->cap_words || n_max > p->cap_req ||
        b->max_len > p->max_len)
        return fail(BSORT_E_CAPACITY, "batch exceeds the plan's capacity");
    if ((st = check_ws(p->lay, ws, ws_bytes)) != BSORT_OK) return st;
    if (b->n_requests == 0) return BSORT_OK;
    hipStream_t s = (hipStream_t)stream;
    Job j = batch_job(p->lay, (char*)ws, p->bd, b, total, perm);
    HIP_TRY(launch_set_job(j, p->job_dev, s));
    HIP_TRY(hipGraphLaunch(p->exec, s));
    return BSORT_OK;
}

void bsort_plan_destroy(bsort_plan* p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->job_dev) (void)hipFree(p->job_dev);
    if (p->fan) {
        fan_destroy(*p->fan);
        delete p->fan;
    }
    delete p;
}

}  // extern "C"

// ---- the entry point that allocates nothing
//
// For callers that cannot allocate (code under graph capture, serving loops,
// harnesses that forbid hipMalloc): the workspace is this file-scope device
// array, one per GPU, held until the process ends.  Its address on each
// device comes from hipGetSymbolAddress on the first call with that device
// current; host code uses only that address (the array's name in host code
// is a stand-in, not a device address).  Every call on a GPU shares the
// array: calls that overlap on one GPU race.  A call clears what must start
// at zero itself (status word, counters), as the workspace calls do.
constexpr size_t kStaticScratchBytes = BSORT_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static hipError_t static_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p || ((uintptr_t)p & 255)) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// the call's device status word (src) to the caller's word; 0 when src is NULL
__global__ void k_status_out(const uint32_t* src, uint32_t* dst) {
    if (threadIdx.x == 0) *dst = src ? *src : 0u;
}

extern "C" {

bsort_status bsort_sort_batch_static(const bsort_batch* b, int32_t* perm, const bsort_tuning* t,
                                     uint32_t* status, bsort_stream_t stream) {
    int64_t total, n_max;
    bsort_status st = check_batch(b, perm, total, n_max);
    if (st != BSORT_OK) return st;
    if ((st = check_tuning(t)) != BSORT_OK) return st;
    if (t && (t->flags & BSORT_FLAG_PER_BUCKET_LAUNCH))
        return fail(BSORT_E_INVALID, "the per-bucket form is not available without allocation");
    Layout L;
    make_layout(total, b->n_requests, b->max_len, L);
    if (L.bytes > kStaticScratchBytes)
        return fail(BSORT_E_WORKSPACE, "the batch needs " + std::to_string(L.bytes) +
                                           " bytes of scratch; the static scratch holds " +
                                           std::to_string(kStaticScratchBytes));
    hipStream_t s = (hipStream_t)stream;
    void* ws = nullptr;
    HIP_TRY(static_scratch(&ws));
    if (b->n_requests > 0) {
        bsort_tuning tt;
        memset(&tt, 0, sizeof(tt));
        if (t) tt = *t;
        tt.flags |= BSORT_FLAG_SERIAL_STAGES;          // no library stream is created
        Bounds bd = make_bounds(L, total, b->n_requests, n_max, &tt);
        bd.fused_pack = 1;
        Job* jd = (Job*)((char*)ws + L.job);
        Job j = batch_job(L, (char*)ws, bd, b, total, perm);
        HIP_TRY(launch_set_job(j, jd, s));
        HIP_TRY(enqueue_sort(jd, bd, s, true, nullptr, nullptr));
    }
    if (status) {
        k_status_out<<<1, 64, 0, s>>>(
            b->n_requests > 0 ? (const uint32_t*)((char*)ws + L.status) : nullptr, status);
        HIP_TRY(hipGetLastError());
    }
    return BSORT_OK;
}

bsort_status bsort_get_device_status(void* ws, bsort_stream_t stream) {
    if (!ws) return fail(BSORT_E_WORKSPACE, "workspace is NULL");
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    uint32_t v = 0;
    HIP_TRY(hipMemcpy(&v, ws, sizeof(v), hipMemcpyDeviceToHost));
    if (v == 0) return BSORT_OK;
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(ws, &zero, sizeof(zero), hipMemcpyHostToDevice));
    std::string what;
    if (v & ST_TOO_LONG) what += " word longer than max_len;";
    if (v & ST_BAD_OFFSETS) what += " offsets decrease or pass n_bytes;";
    if (v & ST_BAD_REQ) what += " request bounds inconsistent;";
    if (v & ST_OVERFLOW) what += " internal list overflow;";
    if (v & ST_STALLED) what += " a wait of the merge-split launch gave up;";
    g_err = "device status:" + what;
    if (v & ST_TOO_LONG) return BSORT_E_TOO_LONG;
    return BSORT_E_INVALID;
}

const char* bsort_status_string(bsort_status s) {
    switch (s) {
        case BSORT_OK: return "ok";
        case BSORT_E_INVALID: return "invalid argument";
        case BSORT_E_TOO_LONG: return "word too long";
        case BSORT_E_NO_MEMORY: return "out of memory";
        case BSORT_E_WORKSPACE: return "workspace too small or misaligned";
        case BSORT_E_HIP: return "HIP runtime error";
        case BSORT_E_CAPACITY: return "batch exceeds plan capacity";
    }
    return "unknown status";
}

const char* bsort_last_error(void) { return g_err.c_str(); }

const char* bsort_version(void) { return "bsort 0.1 gfx950"; }

}  // extern "C"

namespace {

// The plain form: the batched form's kernels, launched per list and per
// sub-array.  Per list, the bucketize launches (the scatter packs the key
// lanes, as in the batched form); one host synchronisation to read every
// sub-array's size and key offset; then per (list, length) sub-array one
// launch routed as the batched plan routes it (one register tile, one in-LDS
// sort, or the chunk sorts of a sub-array merged through HBM) and, for the
// last, one launch per merge-split phase.
bsort_status plain_form(const bsort_batch* b, int32_t* perm, const bsort_tuning* t,
                        const Layout& L, char* ws, hipStream_t s) {
    const int32_t R = b->n_requests;
    const int ml1 = L.ml1;
    const int wmax = L.wmax;
    const int64_t* h = b->h_req_start;
    Job* jobs = (Job*)(ws + L.jobs);
    Bounds bd0 = make_bounds(L, h[R], R, 0, t);
    for (int32_t r = 0; r < R; ++r) {
        const int64_t n = h[r + 1] - h[r];
        Layout Lr;
        make_layout(n, 1, L.ml1 - 1, Lr);
        Bounds br = make_bounds(Lr, n, 1, n, t);
        br.fused_pack = 1;
        Job j = base_job(L, ws, bd0);
        j.bytes = b->bytes;
        j.n_bytes = b->n_bytes;
        j.offsets = b->offsets + h[r];
        j.total = n;
        j.R = 1;
        j.max_len = b->max_len;
        j.rs_inline[0] = 0;
        j.rs_inline[1] = n;
        j.req_start = (const int64_t*)((char*)&jobs[r] + offsetof(Job, rs_inline));
        j.counts = (int32_t*)(ws + L.counts) + (int64_t)r * ml1;
        j.starts = (int32_t*)(ws + L.starts) + (int64_t)r * (ml1 + 1);
        j.order = (int32_t*)(ws + L.order) + h[r];
        j.len8 = (uint8_t*)(ws + L.len8) + h[r];
        j.perm = perm + h[r];
        j.keys = (uint64_t*)(ws + L.keys) + (int64_t)wmax * h[r];
        j.key_off = (int64_t*)(ws + L.key_off) + (int64_t)r * ml1;
        // each list keeps its own chunk map; the chunk histograms are reused
        // in stream order
        j.chunk_begin = (int64_t*)((char*)&jobs[r] + offsetof(Job, cb_inline));
        j.chunk_cap = Lr.chunk_cap;
        j.flags |= kJobFusedPack;
        if (r > 0) j.flags |= kJobKeepStatus;
        HIP_TRY(launch_set_job(j, &jobs[r], s));
        br.chunk_cap = Lr.chunk_cap;
        HIP_TRY(launch_bucketize(&jobs[r], br, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> cnt((size_t)R * ml1), st((size_t)R * (ml1 + 1));
    std::vector<int64_t> ko((size_t)R * ml1);
    HIP_TRY(hipMemcpy(cnt.data(), ws + L.counts, sizeof(int32_t) * cnt.size(),
                      hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st.data(), ws + L.starts, sizeof(int32_t) * st.size(),
                      hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ko.data(), ws + L.key_off, sizeof(int64_t) * ko.size(),
                      hipMemcpyDeviceToHost));
    const bool tiles_only = t && (t->flags & BSORT_FLAG_TILES_ONLY);
    for (int32_t r = 0; r < R; ++r) {
        if (h[r + 1] == h[r]) continue;
        for (int l = 1; l < ml1; ++l) {
            const int nb = cnt[(size_t)r * ml1 + l];
            if (nb < 2) continue;
            const int64_t pos0 = st[(size_t)r * (ml1 + 1) + l];
            const int64_t k0 = ko[(size_t)r * ml1 + l];
            const int D = dwords_for_len(l);
            int c = -1;
            if (nb > bd0.tile_keys[D])
                for (int q = 0; q < kLdsClasses && c < 0; ++q)
                    if (lds_fits(D, q) && nb <= lds_cap(q, D)) c = q;
            if (nb <= bd0.tile_keys[D]) {                  // one register tile
                TileDesc td{pos0, k0, nb, 0, nb, l};
                HIP_TRY(launch_tile_one_bucket(&jobs[r], D, td, 1, nb, false, s));
                continue;
            }
            if (c >= 0) {                                  // the whole sub-array in LDS
                LBucket lb{pos0, k0, nb, l, nb, 0};
                HIP_TRY(launch_lds_one(&jobs[r], D, c, lb, 1, 0, s));
                continue;
            }
            // merged through HBM: chunks (in LDS, or register tiles), then phases
            const int T = bd0.hbm_tile_keys[D];
            const int nt = (nb + T - 1) / T;
            if (D <= kLdsMaxD && bd0.hbm_class[D] >= 0) {
                LBucket lb{pos0, k0, nb, l, nb, 1};
                HIP_TRY(launch_lds_one(&jobs[r], D, bd0.hbm_class[D], lb, nt, T, s));
            } else {
                TileDesc td{pos0, k0, nb, 0, 0, l};
                HIP_TRY(launch_tile_one_bucket(&jobs[r], D, td, nt, T, nt > 1 && !tiles_only, s));
            }
            if (nt < 2 || tiles_only) continue;
            MSub m{pos0, k0, 0, nb, l, T, nt};
            for (int ph = 0; ph < nt; ++ph)
                HIP_TRY(launch_merge_phase_one(&jobs[r], m, ph, bd0.pair_lds, s));
        }
    }
    return BSORT_OK;
}

}  // namespace
