// Host side of the cpmi C ABI: argument checks, workspace, tile lists, the
// launch sequence of one exact search, buffer growth, HIP-graph replay of the
// batched motif search, and the tuned-configuration cache.
//
// One exact search over a set of problems (point sets or series) enqueues:
//   reset -> row prep / window builder -> screen pass 1 (tile minima, radius
//   candidates) -> bound reduction and tile selection -> screen pass 2 on the
//   selected tiles (closest-pair candidates) -> FP64 verification -> result
// and synchronises once. Candidate buffers that overflowed are grown and the
// search is re-run (the screen never writes past a buffer's capacity; its
// counters keep counting, so the size needed is known after one run).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cpmi.h"
#include "bound.h"
#include "cpmi_internal.h"
#include "layout256.h"

using namespace cpmi;

// Device memory of the allocation-free closest pair (cpmi_closest_pair_noalloc):
// one static array per GPU, held until the process ends. Host code never
// passes its name to a kernel or a copy: each device's address is taken once
// with hipGetSymbolAddress (cpmi_create, with the device current) and used
// from then on.
static constexpr size_t kScratchBytes = CPMI_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static void *g_scratch_addr[kMaxDevices];
static std::mutex g_scratch_mu;

namespace {

struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};

constexpr int BAND_DEFAULT = 8;   // block rows per band of the tile order, untuned

// Device memory of one exact search. The context owns one set, grown on
// demand; the allocation-free entry point carves a set out of the static
// scratch array instead (Arena).
struct Work {
    DevBuf xs, shat, bmax, musg, probs, jobs, tiles, tile_min, sel, candR, candU, cand_d2, keys, vals, cnt, ubits, res,
        mrowstat;
};

// Bump allocation over a fixed device range.
struct Arena {
    char *base = nullptr;
    size_t size = 0, used = 0;
};

struct HostProb {
    int64_t n = 0, d = 0, ld = 0;   // rows, dimension, source stride
    int64_t excl = 1;
    int motif = 0;
    int src_i8 = 0;
    double r2 = -1.0;
    const void *src = nullptr;      // points, or the series
    int band = BAND_DEFAULT;        // block rows per band of the tile order
    int64_t len = 0;                // series length (motif)
    int32_t kpad = 0;
    int64_t npad = 0;
    const int32_t *perm = nullptr;  // screen row r holds source row perm[r] (reference-point order), or null
    const int32_t *iperm = nullptr; // its inverse (windows of a series: the builder writes window w to row iperm[w])
    int64_t split = 0;              // two-set problem: first row of the second set (multiple of 256), else 0
    int64_t na = 0;                 // two-set problem: rows of the first set (the second has n - split)
    // workspace offsets
    size_t xs_off = 0, sh_off = 0, bm_off = 0, mu_off = 0;
};

// One autotuner decision: for screens of precision `prec` (P_F32, P_BF16,
// P_I8; 0 = the precision chosen for CPMI_PREC_AUTO on float input) whose
// dimension falls in K bucket `kb` (next power of two >= max(d, 64)) and whose
// size falls in row bucket `rb` (ceil(log2) of the row count, or of the row
// count of a single problem with as many pairs for a batch), `value` is the
// tile edge (128 or 256), or the precision for prec = 0. Entries of kind
// KIND_BAND hold the band height of the tile order (block rows per band) for
// that precision and buckets.
struct TuneEntry {
    int prec, kb, rb, value;
    int kind = 0;
};
enum { KIND_TILE = 0, KIND_BAND = 1 };

// 64-bit device counters: radius candidates, pair candidates, selected tiles,
// verified radius pairs, radius pairs counted by the screen alone
constexpr int NCNT = 5;
enum { C_R = 0, C_U = 1, C_SEL = 2, C_OUT = 3, C_IN = 4 };
// Largest candidate or output buffer a search grows to (entries). A radius
// search whose candidates exceed it is re-run in the counting form, which
// gives the exact number of pairs without storing them.
constexpr uint64_t CAND_MAX = 1ull << 28;
// Radius lists longer than this are sorted by one radix sort; shorter ones by
// the bitonic sort (one launch up to 2,048 pairs).
constexpr int64_t RADIX_SORT_FROM = 1 << 14;

}  // namespace

struct cpmi_ctx {
    int device = 0;
    std::string err;
    cpmi_stats stats{};
    int tile_override[4] = {0, 0, 0, 0};
    int band_override = 0;         // band height forced by the autotuner while it times one
    std::vector<TuneEntry> tuned;  // autotuner results (cache file and cpmi_autotune)

    Work w;  // device memory of the searches (grown on demand)
    uint64_t capR = 1u << 20, capU = 1u << 18, capOut = 1u << 20;

    // host mirrors
    void *pinned = nullptr;  // counters + results read back
    size_t pinned_cap = 0;

    // tile list cache
    std::vector<int64_t> tiles_key;
    int64_t ntiles = 0;
    int64_t nfull = 0;   // leading entries of the list that are full tiles
    int64_t nfull_pairs = 0;  // pairs covered by the timed screen launch (full tiles, or all when none is full)

    void *scratch = nullptr;  // this device's static scratch (device address)
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t es0 = nullptr, es1 = nullptr;  // around the first screen pass
    hipStream_t own = nullptr;
    int ncu = 256;

    // captured batch graph
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> graph_key;

    // reference-point tile pruning of point sets (cpmi_set_pruning)
    int prune_q = 0;
    double prune_f = 10.0;
    uint64_t prune_seed = 0;
    DevBuf mD, mperm, miperm, mlo, mhi, mrefs, msort;
    // the pruned tile list built on the device: entries, per-segment counts
    // and their scan, scan scratch, and its four totals (device; pinned copy)
    DevBuf mtl, mseg, mscan, mout4;
    // neighbour lists (cpmi_pairs_to_csr): keys, counts, offsets; sort scratch
    DevBuf csrW, csrT;
    // radius lists past RADIX_SORT_FROM pairs: sorted keys and values, sort scratch
    DevBuf srtK, srtV, srtT;
    int64_t *plist = nullptr;
    // row order for radius queries with q >= 2: 0 = two references (buckets of
    // the first reference's distance, width prune_w times R, sorted by the
    // second's), 1 = the first reference alone
    int prune_order = 0;
    double prune_w = 1.0;
    // string problems: encoded int8 rows and the encoder's flag word
    DevBuf mZ, mflag;
    // light-bulb bucketing: keys and rows (in, out), sort scratch, columns,
    // candidates, counters
    DevBuf lbA, lbT, lbC, lbP, lbK;
};

namespace {

int fail(cpmi_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(cpmi_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

#define HIPCHK(c, call)                                                                                  \
    do {                                                                                                 \
        hipError_t e_ = (call);                                                                          \
        if (e_ != hipSuccess) return fail((c), CPMI_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

int ensure(cpmi_ctx *c, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (b.cap >= bytes) return CPMI_OK;
    if (b.p) {
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipFree(b.p));
        b.p = nullptr;
        b.cap = 0;
    }
    size_t want = bytes + bytes / 4;
    want = (want + 4095) & ~(size_t)4095;
    HIPCHK(c, hipMalloc(&b.p, want));
    b.cap = want;
    // any captured graph refers to the old addresses
    if (c->gexec) {
        hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        c->graph_key.clear();
    }
    return CPMI_OK;
}

int ensure_pinned(cpmi_ctx *c, size_t bytes)
{
    if (c->pinned_cap >= bytes) return CPMI_OK;
    if (c->pinned) hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_cap = 0;
    HIPCHK(c, hipHostMalloc(&c->pinned, bytes, hipHostMallocDefault));
    c->pinned_cap = bytes;
    return CPMI_OK;
}

int elem_bytes(int prec) { return prec == P_F32 ? 4 : (prec == P_BF16 ? 2 : 1); }

// Rows are padded to 128 bytes: whole LDS slices of the 128-tile screen, and
// pairs of 64-byte slices of the 256-tile screen (whose load ring turns four
// slices at a time; a launch with rows of 4k + 2 slices takes its K2 form).
int32_t kpad_for(int prec, int64_t d, int tile)
{
    (void)tile;
    const int64_t per = 128 / elem_bytes(prec);
    return (int32_t)((d + per - 1) / per * per);
}

// Some problem's rows hold 4k + 2 slices of the 256-tile screen.
bool needs_k2(const std::vector<HostProb> &hp, int prec)
{
    for (const HostProb &h : hp)
        if (((int64_t)h.kpad * elem_bytes(prec) / 64) % 4 != 0) return true;
    return false;
}

const char *prec_name(int prec) { return prec == P_F32 ? "f32" : (prec == P_BF16 ? "bf16" : "i8"); }

int kbucket(int64_t d)
{
    int b = 64;
    while (b < d && b < (1 << 20)) b <<= 1;
    return b;
}

// Row bucket of a problem with `pairs` admissible pairs: ceil(log2) of the row
// count of a single point set with as many pairs.
int rbucket(double pairs)
{
    // n(n-1)/2 = pairs  <=>  n = 1/2 + sqrt(1/4 + 2 pairs)
    const double rows = 0.5 + std::sqrt(0.25 + 2.0 * std::max(pairs, 1.0));
    int r = 0;
    while ((double)(1ll << r) < rows * (1.0 - 1e-12) && r < 40) ++r;
    return std::max(r, 8);
}

int64_t pairs_of(int64_t n, int64_t excl)
{
    const int64_t m = n - excl;
    return m > 0 ? m * (m + 1) / 2 : 0;
}

// Admissible pairs of a problem: i < j with j - i >= excl, or for two sets
// every (first-set row, second-set row) pair but the rows of equal index.
int64_t pairs_of(const HostProb &h)
{
    if (h.split > 0) {
        const int64_t nb = h.n - h.split;
        return h.na * nb - std::min(h.na, nb);
    }
    return pairs_of(h.n, h.excl);
}

// Tuned value for (prec, kb, rb): the exact entry, else the entry of the
// nearest row bucket with the same precision and K bucket (ties: the larger
// bucket), else -1.
int tuned_value(const cpmi_ctx *c, int prec, int kb, int rb, int kind = KIND_TILE)
{
    int best = -1, dist = 1 << 30, brb = -1;
    for (const TuneEntry &e : c->tuned) {
        if (e.kind != kind || e.prec != prec || e.kb != kb) continue;
        const int dd = std::abs(e.rb - rb);
        if (dd < dist || (dd == dist && e.rb > brb)) {
            best = e.value;
            dist = dd;
            brb = e.rb;
        }
    }
    return best;
}

void set_tuned(cpmi_ctx *c, int prec, int kb, int rb, int value, int kind = KIND_TILE)
{
    for (TuneEntry &e : c->tuned)
        if (e.kind == kind && e.prec == prec && e.kb == kb && e.rb == rb) {
            e.value = value;
            return;
        }
    c->tuned.push_back(TuneEntry{prec, kb, rb, value, kind});
}

// Band height of the tile order for one problem of dimension d with `pairs`
// admissible pairs at precision prec: the override, the tuned choice, or 8.
int pick_band(const cpmi_ctx *c, int prec, int64_t d, double pairs)
{
    if (c->band_override > 0) return c->band_override;
    const int v = tuned_value(c, prec, kbucket(d), rbucket(pairs), KIND_BAND);
    return v >= 1 && v <= 64 ? v : BAND_DEFAULT;
}

// Screen tile for a problem of dimension d (the largest, for a batch) and
// `pairs` admissible pairs: the override, else the tuned choice, else 256 when
// the 256-tiles are enough to keep every CU busy several times over and 128
// otherwise.
int pick_tile(cpmi_ctx *c, int prec, int64_t d, double pairs)
{
    if (c->tile_override[prec]) return c->tile_override[prec];
    const int v = tuned_value(c, prec, kbucket(d), rbucket(pairs));
    if (v == 128 || v == 256) return v;
    return pairs / (256.0 * 256.0) >= 4.0 * c->ncu ? 256 : 128;
}

const char *tune_name(int prec) { return prec == 0 ? "auto" : prec_name(prec); }

// Reader of the tuner's JSON object {"bf16:k512:r18": 256, "auto:k512:r18": 2, ...}.
// Unknown or malformed entries are ignored.
void load_tune_cache(cpmi_ctx *c, const char *path)
{
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    fclose(f);
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        size_t e = s.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string key = s.substr(pos + 1, e - pos - 1);
        pos = e + 1;
        size_t colon = s.find_first_not_of(" \t\r\n", e + 1);
        if (colon == std::string::npos || s[colon] != ':') continue;
        char *end = nullptr;
        const long v = strtol(s.c_str() + colon + 1, &end, 10);
        if (end == s.c_str() + colon + 1) continue;
        char name[24] = {0};
        int kb = 0, rb = 0;
        if (sscanf(key.c_str(), "%23[a-z0-9.]:k%d:r%d", name, &kb, &rb) != 3) continue;
        int kind = KIND_TILE;
        const char *pn = name;
        if (!strncmp(name, "band.", 5)) {
            kind = KIND_BAND;
            pn = name + 5;
        }
        int prec = -1;
        for (int p = 0; p <= 3; ++p)
            if (!strcmp(pn, tune_name(p))) prec = p;
        if (prec < 0 || kb < 64 || kb > (1 << 20) || rb < 0 || rb > 40) continue;
        if (kind == KIND_BAND) {
            if (prec == 0 || v < 1 || v > 64) continue;
        } else if (prec == 0 ? (v != P_F32 && v != P_BF16) : (v != 128 && v != 256)) {
            continue;
        }
        set_tuned(c, prec, kb, rb, (int)v, kind);
    }
}

// Tile list: upper-triangle tiles holding at least one admissible pair. The
// list holds first the full tiles (every pair admissible) and then the partial
// ones (diagonal, exclusion band, ragged edge); *nfull counts the former. For
// a single problem the tiles are ordered in bands of 8 tile rows
// (column-major in a band, so concurrent work-groups share row and column
// panels) and the full part is split into 8 contiguous chunks interleaved
// slot by slot, so that the work-groups the dispatcher sends to one XCD
// (slot % 8) walk one chunk and keep its panels in that XCD's L2. For several
// problems (uneven costs) the tiles are listed most-expensive problem first,
// each problem's full tiles chunked and interleaved the same way.
// keep(I, J) (optional, single problem) drops tiles proved empty of answers;
// jend[I] (optional) is a block column from which on every tile of row I is
// dropped, so that the scan of a band can stop there. For the windows of a
// series in reference order (perm set) screen rows are not positions: every
// tile may hold excluded pairs, so all are partial.
void build_tiles(const std::vector<HostProb> &hp, int tile, std::vector<uint64_t> &out, int64_t *nfull,
                 const std::function<bool(int64_t, int64_t)> &keep = {}, const std::vector<int64_t> *jend = nullptr)
{
    std::vector<uint64_t> L, part;
    std::vector<size_t> runs;   // several problems: where each problem's full tiles start in L
    std::vector<size_t> order(hp.size());
    for (size_t p = 0; p < hp.size(); ++p) order[p] = p;
    if (hp.size() > 1)
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
            return hp[a].kpad > hp[b].kpad || (hp[a].kpad == hp[b].kpad && hp[a].n > hp[b].n);
        });
    for (size_t oi = 0; oi < hp.size(); ++oi) {
        const size_t p = order[oi];
        const HostProb &h = hp[p];
        const int64_t G = std::max(1, h.band);
        if (pairs_of(h) == 0) continue;
        runs.push_back(L.size());
        const bool permuted = h.motif && h.perm;
        const int64_t nT = (h.n + tile - 1) / tile;
        if (h.split > 0) {
            // two sets: block rows of the first set against block columns of
            // the second, in bands of G rows (column-major in a band); a tile
            // is partial on the ragged edges and where row i meets column
            // split + i
            const int64_t nA = (h.na + tile - 1) / tile, J0 = h.split / tile;
            for (int64_t b0 = 0; b0 < nA; b0 += G)
                for (int64_t J = J0; J < nT; ++J)
                    for (int64_t I = b0; I < std::min(b0 + G, nA); ++I) {
                        // rows i in [r0, r1), second-set indices j - split in [c0, c1):
                        // no admissible pair if every pair is an equal-index one
                        const int64_t r0 = I * tile, r1 = std::min((I + 1) * tile, h.na);
                        const int64_t c0 = J * tile - h.split, c1 = std::min((J + 1) * tile, h.n) - h.split;
                        const int64_t same = std::max<int64_t>(0, std::min(r1, c1) - std::max(r0, c0));
                        if ((r1 - r0) * (c1 - c0) == same) continue;
                        if (keep && !keep(I, J)) continue;
                        const bool full = ((I + 1) * tile <= h.na) && ((J + 1) * tile <= h.n) && (J - J0 != I);
                        (full ? L : part).push_back(tile_pack((uint32_t)p, (uint32_t)I, (uint32_t)J));
                    }
            continue;
        }
        for (int64_t b0 = 0; b0 < nT; b0 += G) {
            int64_t jstop = nT;
            if (jend) {
                jstop = 0;
                for (int64_t I = b0; I < std::min(b0 + G, nT); ++I) jstop = std::max(jstop, (*jend)[I]);
            }
            for (int64_t J = b0; J < jstop; ++J)
                for (int64_t I = b0; I < std::min(b0 + G, nT) && I <= J; ++I) {
                    const int64_t maxj = std::min(J * tile + tile - 1, h.n - 1);
                    if (!permuted && maxj - I * tile < h.excl) continue;
                    if (keep && !keep(I, J)) continue;
                    const bool full = !permuted && (J * tile - (I * tile + tile - 1) >= h.excl) &&
                                      ((I + 1) * tile <= h.n) && ((J + 1) * tile <= h.n);
                    (full ? L : part).push_back(tile_pack((uint32_t)p, (uint32_t)I, (uint32_t)J));
                }
        }
    }
    // each problem's full tiles split into 8 contiguous chunks interleaved
    // slot by slot (its run padded to a whole number of 8 slots, so that slot
    // s of every run goes to XCD s % 8): every XCD walks an eighth of every
    // problem, in band order
    out.clear();
    runs.push_back(L.size());
    for (size_t r = 0; r + 1 < runs.size(); ++r) {
        const int64_t a = (int64_t)runs[r], T = (int64_t)runs[r + 1] - a;
        const int64_t C = (T + 7) / 8, base = (int64_t)out.size();
        out.resize(base + C * 8, TILE_NONE);
        for (int64_t s = 0; s < C * 8; ++s) {
            const int64_t src = (s % 8) * C + s / 8;
            if (src < T) out[base + s] = L[a + src];
        }
    }
    *nfull = (int64_t)out.size();
    out.insert(out.end(), part.begin(), part.end());
}

// A tile list built on the device: the entries (8 bytes each), how many, how
// many leading slots hold full tiles, and the tiles of the timed launch.
struct DevList {
    const uint64_t *tiles;
    int64_t ntiles, nfull, timed_tiles;
};

// Test of the screen bound (cpmi_dbg_screen_sample): device buffers of the
// dumped screen values, canonical d2, per-tile bounds and the largest ratio.
struct DumpReq {
    void *out;
    double *d2;
    double *E;
    unsigned int *ratio;
};

struct RunOut {
    std::vector<ResDev> res;
    uint64_t cnt[NCNT];
    bool counted = false;   // radius search ran in the counting form: pairs not stored
    // pairs within the radius (exact)
    uint64_t radius_pairs() const { return cnt[C_OUT] + (counted ? cnt[C_IN] : 0); }
};

// Slice of `bytes` of the arena for b (no allocation).
int take(cpmi_ctx *c, Arena &ar, DevBuf &b, size_t bytes)
{
    if (b.p && b.cap >= bytes) return CPMI_OK;
    const size_t want = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    if (ar.used + want > ar.size)
        return fail(c, CPMI_ERR_CAPACITY, "the search needs more than the %zu bytes of static scratch", ar.size);
    b.p = ar.base + ar.used;
    b.cap = want;
    ar.used += want;
    return CPMI_OK;
}

// Launch the whole exact search for the problems in hp; synchronises once.
// `forced` (optional) is a tile list built by the caller (reference-point
// pruning) with its first `forced_nfull` entries full tiles; it bypasses the
// list cache. `reuse_operand` skips the row preparation: the screen operand
// and row scalars of the previous call (same problems, precision and tile)
// are still in the workspace. With an arena, every device buffer is a slice
// of it (nothing is allocated; a search that does not fit fails with
// CPMI_ERR_CAPACITY) and the context's workspace and list cache are untouched.
int run_search(cpmi_ctx *c, std::vector<HostProb> &hp, int prec, int tile, bool want_cpp, bool want_frnn,
               hipStream_t st, bool batch_graph, RunOut &ro, const std::vector<uint64_t> *forced = nullptr,
               int64_t forced_nfull = 0, bool reuse_operand = false, const std::function<void()> &while_busy = {},
               Arena *ar = nullptr, const DumpReq *dump = nullptr, const DevList *dlist = nullptr)
{
    bool busy_done = false;
    Work local;
    Work &W = ar ? local : c->w;
    auto get = [&](DevBuf &b, size_t bytes) { return ar ? take(c, *ar, b, bytes) : ensure(c, b, bytes); };
    const int64_t np = (int64_t)hp.size();
    const int esz = elem_bytes(prec);
    // ---- workspace layout
    size_t xs_b = 0, sh_b = 0, bm_b = 0, mu_b = 0;
    for (auto &h : hp) {
        h.kpad = kpad_for(prec, h.d, tile);
        h.npad = (h.n + 255) / 256 * 256;
        h.xs_off = xs_b;
        xs_b += (size_t)h.npad * h.kpad * esz;
        h.sh_off = sh_b;
        sh_b += (size_t)h.npad * 4;
        h.bm_off = bm_b;
        bm_b += (size_t)(h.npad / tile) * sizeof(float4);
        h.mu_off = mu_b;
        if (h.motif) mu_b += (size_t)h.npad * 8;
    }
    int rc;
    if ((rc = get(W.xs, xs_b))) return rc;
    // BF16: the folded row scalars (8 bytes a row) follow the row scalars
    const size_t fold_b = prec == P_BF16 ? 2 * sh_b : 0;
    if ((rc = get(W.shat, sh_b + fold_b))) return rc;
    if ((rc = get(W.bmax, bm_b))) return rc;
    if ((rc = get(W.musg, 2 * mu_b))) return rc;
    if ((rc = get(W.probs, np * sizeof(Prob)))) return rc;
    if ((rc = get(W.res, np * sizeof(ResDev)))) return rc;
    if ((rc = get(W.ubits, np * 8))) return rc;
    if ((rc = get(W.cnt, NCNT * 8))) return rc;

    // ---- tile list (cached by shape)
    std::vector<int64_t> key{(int64_t)tile, np};
    for (auto &h : hp) {
        h.band = pick_band(c, prec, h.d, (double)pairs_of(h));
        key.push_back(h.band);
        key.push_back(h.n);
        key.push_back(h.excl);
        key.push_back(h.kpad);
        key.push_back(h.split);
        key.push_back(h.na);
    }
    // pairs of the timed launch: the full tiles, or every tile when all are partial
    auto timed_pairs = [&](const std::vector<uint64_t> &tl, int64_t nf) {
        const int64_t nt = nf > 0 ? nf : (int64_t)tl.size();
        int64_t nreal = 0;
        for (int64_t k = 0; k < nt; ++k) nreal += tl[k] != TILE_NONE;
        return nreal * (int64_t)tile * tile;
    };
    // the screen kernels index the tile list with 32-bit integers
    auto list_fits = [&]() {
        double est = 0.0;
        for (auto &h : hp) {
            const double nT = std::ceil((double)h.n / tile);
            est += nT * (nT + 1.0) / 2.0;
        }
        if (est > 2147483647.0 - 1048576.0)
            return fail(c, CPMI_ERR_ARG, "problem too large for one screen (%.3g tiles; at most 2^31)", est);
        return (int)CPMI_OK;
    };
    int64_t ntiles, nfull, nfull_pairs;
    if (dlist) {
        // a list the device built (reference-point pruning): copied into place
        ntiles = dlist->ntiles;
        nfull = dlist->nfull;
        nfull_pairs = dlist->timed_tiles * (int64_t)tile * tile;
        if ((rc = get(W.tiles, std::max<size_t>(ntiles, 1) * 8))) return rc;
        if ((rc = get(W.tile_min, std::max<size_t>(ntiles, 1) * 16))) return rc;
        if ((rc = get(W.sel, std::max<size_t>(ntiles, 1) * 16))) return rc;
        if (ntiles > 0)
            HIPCHK(c, hipMemcpyAsync(W.tiles.p, dlist->tiles, ntiles * 8, hipMemcpyDeviceToDevice, st));
        if (!ar) c->tiles_key.clear();
    } else if (forced || ar) {
        std::vector<uint64_t> built;
        if (!forced) {
            if ((rc = list_fits())) return rc;
            build_tiles(hp, tile, built, &forced_nfull);
        }
        const std::vector<uint64_t> &tl = forced ? *forced : built;
        nfull = forced_nfull;
        nfull_pairs = timed_pairs(tl, forced_nfull);
        if ((rc = get(W.tiles, std::max<size_t>(tl.size(), 1) * 8))) return rc;
        if ((rc = get(W.tile_min, std::max<size_t>(tl.size(), 1) * 16))) return rc;
        if ((rc = get(W.sel, std::max<size_t>(tl.size(), 1) * 16))) return rc;
        if (!tl.empty()) HIPCHK(c, hipMemcpyAsync(W.tiles.p, tl.data(), tl.size() * 8, hipMemcpyHostToDevice, st));
        if (!tl.empty() && !forced) HIPCHK(c, hipStreamSynchronize(st));   // `built` is released on return
        ntiles = (int64_t)tl.size();
        if (!ar) c->tiles_key.clear();  // the cached list is gone
    } else {
        if (key != c->tiles_key) {
            if ((rc = list_fits())) return rc;
            std::vector<uint64_t> tl;
            int64_t nf = 0;
            build_tiles(hp, tile, tl, &nf);
            c->nfull = nf;
            c->nfull_pairs = timed_pairs(tl, nf);
            if ((rc = get(W.tiles, tl.size() * 8))) return rc;
            if ((rc = get(W.tile_min, tl.size() * 16))) return rc;
            if ((rc = get(W.sel, tl.size() * 16))) return rc;
            if (!tl.empty()) HIPCHK(c, hipMemcpy(W.tiles.p, tl.data(), tl.size() * 8, hipMemcpyHostToDevice));
            c->ntiles = (int64_t)tl.size();
            c->tiles_key = key;
        }
        ntiles = c->ntiles;
        nfull = c->nfull;
        nfull_pairs = c->nfull_pairs;
    }
    // candidate and output capacities: the context's (grown on overflow), or
    // what the arena has left (closest pair only: no radius buffers)
    uint64_t capR = c->capR, capU = c->capU, capOut = c->capOut;
    if (ar) {
        if (want_frnn) return fail(c, CPMI_ERR_ARG, "the allocation-free search takes no radius");
        capR = capOut = 0;
        const size_t room = ar->size > ar->used + 6 * 256 ? ar->size - ar->used - 6 * 256 : 0;
        capU = std::min<uint64_t>(1u << 20, room / (sizeof(Cand) + 8));
        if (capU < 1024) return fail(c, CPMI_ERR_CAPACITY, "the static scratch has no room left for candidates");
    }
    bool count_mode = false;

    for (int attempt = 0; attempt < 4; ++attempt) {
        if ((rc = get(W.candR, (size_t)capR * sizeof(Cand)))) return rc;
        if ((rc = get(W.candU, (size_t)capU * sizeof(Cand)))) return rc;
        if ((rc = get(W.cand_d2, (size_t)capU * 8))) return rc;
        if ((rc = get(W.keys, (size_t)capOut * 8))) return rc;
        if ((rc = get(W.vals, (size_t)capOut * 8))) return rc;

        // ---- problem descriptors
        std::vector<Prob> P(np);
        std::vector<SeriesJob> jobs;
        int64_t blk = 0;
        for (int64_t p = 0; p < np; ++p) {
            const HostProb &h = hp[p];
            Prob &q = P[p];
            memset(&q, 0, sizeof q);
            q.xs = (char *)W.xs.p + h.xs_off;
            q.shat = (char *)W.shat.p + h.sh_off;
            q.fold = fold_b ? (const uint2 *)((char *)W.shat.p + sh_b + 2 * h.sh_off) : nullptr;
            q.bmax = (const float4 *)((char *)W.bmax.p + h.bm_off);
            q.src = h.src;
            q.n = h.n;
            q.d = h.d;
            q.ld = h.ld;
            q.kpad = h.kpad;
            q.excl = (int32_t)h.excl;
            q.motif = h.motif;
            q.src_i8 = h.src_i8;
            q.r2 = h.r2;
            // the 256-row screen folds the row scalars into the matrix product
            q.form = (tile == 256 && prec != P_I8) ? SCREEN_FOLDED : SCREEN_EPILOGUE;
            q.perm = h.perm;
            q.split = (int32_t)h.split;
            q.na = h.na;
            // each row's own bound terms: for the radius verifier's per-pair
            // bound (one problem with a radius, FP32 / BF16), and for windows
            // in reference order (reduced per block)
            q.rowstat = nullptr;
            if (np == 1 && ((h.r2 >= 0.0 && prec != P_I8) || h.iperm)) {
                if ((rc = get(W.mrowstat, (size_t)h.npad * sizeof(float4)))) return rc;
                q.rowstat = (const float4 *)W.mrowstat.p;
            }
            if (h.motif) {
                q.mu = (const double *)((char *)W.musg.p + h.mu_off);
                q.sigma = (const double *)((char *)W.musg.p + mu_b + h.mu_off);
                SeriesJob j;
                memset(&j, 0, sizeof j);
                j.T = (const float *)h.src;
                j.len = h.len;
                j.ell = h.d;
                j.npad = h.npad;
                j.blk_base = blk;
                blk += h.npad / SERIES_WPB;
                j.xs = (void *)q.xs;
                j.shat = (void *)q.shat;
                j.fold = (uint2 *)q.fold;
                j.bmax = (float4 *)q.bmax;
                j.mu = (double *)q.mu;
                j.sigma = (double *)q.sigma;
                j.flags = &((ResDev *)W.res.p)[p].flags;
                j.kpad = h.kpad;
                j.iperm = h.iperm;
                j.rowstat = (float4 *)q.rowstat;
                jobs.push_back(j);
            }
        }
        HIPCHK(c, hipMemcpyAsync(W.probs.p, P.data(), np * sizeof(Prob), hipMemcpyHostToDevice, st));
        if (!jobs.empty()) {
            if ((rc = get(W.jobs, jobs.size() * sizeof(SeriesJob)))) return rc;
            HIPCHK(c, hipMemcpyAsync(W.jobs.p, jobs.data(), jobs.size() * sizeof(SeriesJob), hipMemcpyHostToDevice,
                                     st));
        }

        const Prob *dprobs = (const Prob *)W.probs.p;
        ResDev *dres = (ResDev *)W.res.p;
        u64c *dcnt = (u64c *)W.cnt.p;
        auto enqueue = [&]() {
            launch_reset_res(dres, np, st);
            launch_fill_u64((uint64_t *)dcnt, 0ull, NCNT, st);
            launch_fill_u64((uint64_t *)W.ubits.p, 0x7ff0000000000000ull, np, st);
            if (reuse_operand) {
                // the operand, row scalars and block maxima are in place
            } else if (!jobs.empty()) {
                launch_fill_u32((uint32_t *)W.bmax.p, 0u, (int64_t)(bm_b / 4), st);
                launch_prep_series((const SeriesJob *)W.jobs.p, (int64_t)jobs.size(), blk, prec, tile, st);
                // windows in reference order (one series): block maxima from the per-row terms
                if (jobs.size() == 1 && jobs[0].iperm)
                    launch_block_max(jobs[0].rowstat, hp[0].npad, tile, (float4 *)P[0].bmax, st);
            } else {
                launch_fill_u32((uint32_t *)W.bmax.p, 0u, (int64_t)(bm_b / 4), st);
                const HostProb &h = hp[0];
                launch_prep_points(h.src, h.src_i8 ? CPMI_I8 : CPMI_F32, h.n, h.d, h.ld, prec, P[0].xs ? (void *)P[0].xs : nullptr,
                                   h.kpad, h.npad, (void *)P[0].shat, (float4 *)P[0].bmax, tile, &dres[0].flags,
                                   h.perm, (uint2 *)P[0].fold, (float4 *)P[0].rowstat, st);
            }
            ScreenArgs a;
            memset(&a, 0, sizeof a);
            a.probs = dprobs;
            a.tiles = (const uint64_t *)W.tiles.p;
            a.ntiles = ntiles;
            a.k2 = tile == 256 && needs_k2(hp, prec);
            if (dump) {
                // the listed tiles' screen values, checked against the canonical d2
                ScreenArgs q = a;
                q.dump = dump->out;
                launch_fill_u32(dump->ratio, 0u, 1, st);
                launch_screen(prec, tile, M_DUMP, true, q, std::min<int64_t>(ntiles, tile == 256 ? c->ncu : 2048), st);
                launch_sample_check(dprobs, a.tiles, ntiles, tile, dump->out, prec, dump->d2, dump->E, dump->ratio, st);
                return;
            }
            a.tile_min = (uint32_t *)W.tile_min.p;
            a.candR = (Cand *)W.candR.p;
            a.cntR = dcnt + C_R;
            a.capR = capR;
            a.candU = (Cand *)W.candU.p;
            a.cntU = dcnt + C_U;
            a.capU = capU;
            a.cntIn = count_mode ? dcnt + C_IN : nullptr;
            // the events bracket the dominant launch: the full-tile screen
            // (the masked one when every tile is partial, and the single
            // masked screen of the 128 tile)
            if (tile == 256) {
                const bool timed_masked = nfull == 0;
                ScreenArgs q = a;
                q.tiles = a.tiles + nfull;
                q.tile_min = a.tile_min + 4 * nfull;
                q.ntiles = ntiles - nfull;
                if (!batch_graph && timed_masked) hipEventRecord(c->es0, st);
                launch_screen(prec, tile, M_MIN, true, q, std::min<int64_t>(ntiles - nfull, c->ncu), st);
                ScreenArgs f = a;
                f.ntiles = nfull;
                if (!batch_graph && !timed_masked) hipEventRecord(c->es0, st);
                launch_screen(prec, tile, M_MIN, false, f, std::min<int64_t>(nfull, c->ncu), st);
                if (!batch_graph) hipEventRecord(c->es1, st);
            } else {
                if (!batch_graph) hipEventRecord(c->es0, st);
                launch_screen(prec, tile, M_MIN, true, a, ntiles, st);
                if (!batch_graph) hipEventRecord(c->es1, st);
            }
            unsigned long long *ubits = want_cpp ? (unsigned long long *)W.ubits.p : nullptr;
            if (want_cpp) launch_reduce_U(dprobs, a.tiles, ntiles, a.tile_min, prec, ubits, st);
            // selected tiles: appended at sel, and in list order at sel + ntiles
            uint64_t *sel = (uint64_t *)W.sel.p;
            launch_select(dprobs, a.tiles, ntiles, a.tile_min, prec, ubits, sel, dcnt + C_SEL, sel + ntiles, st);
            ScreenArgs b = a;
            b.tiles = sel;
            b.sel_count = dcnt + C_SEL;
            b.sel_dense = sel + ntiles;
            b.U = (const double *)ubits;
            launch_screen(prec, tile, M_EMIT, true, b,
                          std::min<int64_t>(std::max<int64_t>(ntiles, 1), tile == 256 ? c->ncu : 2048), st);
            // windows: terms with two divisions each, usually few candidates
            const bool windows = hp[0].motif != 0;
            if (want_cpp) {
                if (windows)
                    launch_verify_windows(false, dprobs, (const Cand *)W.candU.p, dcnt + C_U, capU, prec, tile,
                                          (double *)W.cand_d2.p, nullptr, nullptr, nullptr, 0, dres, st);
                else
                    launch_verify_cpp(dprobs, (const Cand *)W.candU.p, dcnt + C_U, capU, prec, tile,
                                      (double *)W.cand_d2.p, dres, st);
                launch_pick_cpp(dprobs, (const Cand *)W.candU.p, dcnt + C_U, capU, (const double *)W.cand_d2.p,
                                dres, st);
            }
            if (want_frnn) {
                if (windows)
                    launch_verify_windows(true, dprobs, (const Cand *)W.candR.p, dcnt + C_R, capR, prec, tile,
                                          nullptr, (uint64_t *)W.keys.p, (double *)W.vals.p, dcnt + C_OUT,
                                          count_mode ? 0 : capOut, dres, st);
                else
                    launch_verify_frnn(dprobs, (const Cand *)W.candR.p, dcnt + C_R, capR, prec, tile,
                                       (uint64_t *)W.keys.p, (double *)W.vals.p, dcnt + C_OUT,
                                       count_mode ? 0 : capOut, dres, st);
            }
        };

        HIPCHK(c, hipEventRecord(c->ev0, st));
        if (batch_graph) {
            std::vector<int64_t> gkey = key;
            gkey.push_back(prec);
            gkey.push_back((int64_t)capR);
            gkey.push_back((int64_t)capU);
            gkey.push_back((int64_t)capOut);
            gkey.push_back((int64_t)count_mode);
            if (!c->gexec || gkey != c->graph_key) {
                if (c->gexec) {
                    hipGraphExecDestroy(c->gexec);
                    c->gexec = nullptr;
                }
                hipGraph_t g = nullptr;
                HIPCHK(c, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                enqueue();
                hipError_t e = hipStreamEndCapture(st, &g);
                if (e != hipSuccess) return fail(c, CPMI_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
                e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
                hipGraphDestroy(g);
                if (e != hipSuccess) {
                    c->gexec = nullptr;
                    return fail(c, CPMI_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
                }
                c->graph_key = gkey;
            }
            HIPCHK(c, hipGraphLaunch(c->gexec, st));
        } else {
            enqueue();
        }
        HIPCHK(c, hipGetLastError());
        // results and counters: into pinned memory, or (arena) pageable memory
        const size_t rb = np * sizeof(ResDev) + NCNT * 8;
        std::vector<unsigned char> pageable;
        unsigned char *hostbuf;
        if (ar) {
            pageable.resize(rb);
            hostbuf = pageable.data();
        } else {
            if ((rc = ensure_pinned(c, rb))) return rc;
            hostbuf = (unsigned char *)c->pinned;
        }
        HIPCHK(c, hipMemcpyAsync(hostbuf, W.res.p, np * sizeof(ResDev), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(hostbuf + np * sizeof(ResDev), W.cnt.p, NCNT * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipEventRecord(c->ev1, st));
        // host work that overlaps the search (once, not on reruns)
        if (while_busy && !busy_done) {
            busy_done = true;
            while_busy();
        }
        HIPCHK(c, hipStreamSynchronize(st));
        float ms = 0.f;
        hipEventElapsedTime(&ms, c->ev0, c->ev1);
        c->stats.kernel_ms = ms;
        ms = 0.f;
        // (the screen events are not recorded in graph replays and test dumps;
        // a failed query must not leave an error behind for the caller's next call)
        if (!batch_graph && !dump && hipEventElapsedTime(&ms, c->es0, c->es1) != hipSuccess) {
            ms = 0.f;
            (void)hipGetLastError();
        }
        c->stats.screen_ms = ms;
        ro.res.assign((ResDev *)hostbuf, (ResDev *)hostbuf + np);
        memcpy(ro.cnt, hostbuf + np * sizeof(ResDev), sizeof ro.cnt);
        ro.counted = count_mode;

        // a flagged input makes the candidate counts meaningless; report, don't grow
        bool flagged = false;
        for (auto &r : ro.res) flagged |= r.flags != 0;
        auto grown = [](uint64_t need) { return std::min<uint64_t>(need + need / 2 + 1024, CAND_MAX); };
        bool again = false;
        if (!flagged && ro.cnt[C_U] > capU) {
            if (ar || ro.cnt[C_U] > CAND_MAX)
                return fail(c, CPMI_ERR_CAPACITY, "%llu closest-pair candidates (at most %llu)",
                            (unsigned long long)ro.cnt[C_U], (unsigned long long)(ar ? capU : CAND_MAX));
            capU = c->capU = grown(ro.cnt[C_U]);
            again = true;
        }
        if (!flagged && ro.cnt[C_R] > capR) {
            if (ro.cnt[C_R] > CAND_MAX && !count_mode) {
                // too many to store: count the pairs instead (the band of
                // uncertain ones is verified, the rest proved by the screen)
                count_mode = true;
            } else if (ro.cnt[C_R] > CAND_MAX) {
                return fail(c, CPMI_ERR_CAPACITY,
                            "%llu radius candidates within the screening bound of R2 (at most %llu)",
                            (unsigned long long)ro.cnt[C_R], (unsigned long long)CAND_MAX);
            } else {
                capR = c->capR = grown(ro.cnt[C_R]);
            }
            again = true;
        }
        if (!flagged && !count_mode && ro.cnt[C_OUT] > capOut && ro.cnt[C_OUT] <= CAND_MAX) {
            capOut = c->capOut = grown(ro.cnt[C_OUT]);
            again = true;
        }
        if (again) {
            c->stats.reruns++;
            continue;
        }
        c->stats.tiles_total = ntiles;
        c->stats.tiles_rescreened = ro.cnt[C_SEL];
        c->stats.cpp_candidates = ro.cnt[C_U];
        c->stats.frnn_candidates = ro.cnt[C_R];
        c->stats.frnn_pairs = (int64_t)ro.radius_pairs();
        c->stats.precision = prec;
        c->stats.tile = tile;
        int64_t vp = 0;
        for (auto &h : hp) vp += pairs_of(h);
        c->stats.valid_pairs = vp;
        c->stats.screen_pairs = tile == 256 ? nfull_pairs : vp;
        float mr = 0.f;
        for (auto &r : ro.res) mr = std::max(mr, __builtin_bit_cast(float, r.ratio_bits));
        c->stats.max_err_over_bound = mr;
        return CPMI_OK;
    }
    return fail(c, CPMI_ERR_HIP, "candidate buffers kept overflowing");
}

int flags_error(cpmi_ctx *c, uint32_t f)
{
    if (f & F_NONFINITE) return fail(c, CPMI_ERR_NONFINITE, "input holds NaN or Inf");
    if (f & F_DEGENERATE) return fail(c, CPMI_ERR_DEGENERATE, "a window has zero variance");
    if (f & F_RANGE) return fail(c, CPMI_ERR_RANGE, "a squared norm is too large for the FP32 screen");
    return CPMI_OK;
}

void fill_pair(const ResDev &r, cpmi_pair *out)
{
    memset(out, 0, sizeof *out);
    if (r.best_d2 == ~0ull || r.best_ij == ~0ull) {
        out->i = out->j = -1;
        out->status = CPMI_ERR_NOPAIR;
        return;
    }
    out->i = (int64_t)(r.best_ij >> 32);
    out->j = (int64_t)(r.best_ij & 0xffffffffu);
    memcpy(&out->d2, &r.best_d2, 8);
    out->d = std::sqrt(out->d2);
    out->screen_err = __builtin_bit_cast(float, r.err_bits);
    out->screen_bound = __builtin_bit_cast(float, r.bound_bits);
    out->status = CPMI_OK;
}

// Sort the verified radius pairs and copy them to the caller.
int finish_frnn(cpmi_ctx *c, const RunOut &ro, hipStream_t st, int64_t *pairs, double *d2, int64_t cap,
                int64_t *count_out)
{
    const uint64_t count = ro.radius_pairs();
    if (count_out) *count_out = (int64_t)count;
    if ((int64_t)count > cap)
        return fail(c, CPMI_ERR_CAPACITY, "%llu pairs within the radius, capacity %lld", (unsigned long long)count,
                    (long long)cap);
    if (ro.counted || count > CAND_MAX)
        return fail(c, CPMI_ERR_CAPACITY, "%llu pairs within the radius: more than one call returns (%llu)",
                    (unsigned long long)count, (unsigned long long)CAND_MAX);
    if (count == 0) return CPMI_OK;
    int64_t mpad = 1;
    while (mpad < (int64_t)count) mpad <<= 1;
    if ((size_t)mpad * 8 > c->w.keys.cap || (size_t)mpad * 8 > c->w.vals.cap) {
        // grow while keeping the verified pairs
        DevBuf nk, nv;
        HIPCHK(c, hipMalloc(&nk.p, mpad * 8));
        HIPCHK(c, hipMalloc(&nv.p, mpad * 8));
        HIPCHK(c, hipMemcpyAsync(nk.p, c->w.keys.p, (size_t)count * 8, hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipMemcpyAsync(nv.p, c->w.vals.p, (size_t)count * 8, hipMemcpyDeviceToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
        hipFree(c->w.keys.p);
        hipFree(c->w.vals.p);
        c->w.keys.p = nk.p;
        c->w.keys.cap = mpad * 8;
        c->w.vals.p = nv.p;
        c->w.vals.cap = mpad * 8;
        if (c->gexec) {
            hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
            c->graph_key.clear();
        }
    }
    const uint64_t *sk = (const uint64_t *)c->w.keys.p;
    const double *sv = (const double *)c->w.vals.p;
    if ((int64_t)count > RADIX_SORT_FROM) {
        // long lists: one radix sort, out of place
        size_t tb = 0;
        HIPCHK(c, sort_pairs_radix(nullptr, &tb, nullptr, nullptr, nullptr, nullptr, (int64_t)count, st));
        int rc;
        if ((rc = ensure(c, c->srtK, (size_t)count * 8))) return rc;
        if ((rc = ensure(c, c->srtV, (size_t)count * 8))) return rc;
        if ((rc = ensure(c, c->srtT, std::max<size_t>(tb, 1)))) return rc;
        HIPCHK(c, sort_pairs_radix(c->srtT.p, &tb, sk, (uint64_t *)c->srtK.p, sv, (double *)c->srtV.p,
                                   (int64_t)count, st));
        sk = (const uint64_t *)c->srtK.p;
        sv = (const double *)c->srtV.p;
    } else {
        launch_sort_pairs((uint64_t *)c->w.keys.p, (double *)c->w.vals.p, count, mpad, st);
    }
    launch_emit_pairs(sk, sv, count, pairs, d2, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    return CPMI_OK;
}

// Screen precision of a call; AUTO on float input takes the tuned choice for
// the shape (dimension d, `pairs` admissible pairs), else BF16.
int resolve_prec(cpmi_ctx *c, int dtype, int precision, int64_t d, double pairs)
{
    if (dtype == CPMI_I8) {
        if (precision == CPMI_PREC_AUTO || precision == CPMI_PREC_I8) return P_I8;
        return fail(c, CPMI_ERR_ARG, "int8 points take CPMI_PREC_I8 (or AUTO)");
    }
    if (precision == CPMI_PREC_AUTO) {
        const int v = tuned_value(c, 0, kbucket(d), rbucket(pairs));
        return v == P_F32 ? P_F32 : P_BF16;
    }
    if (precision == CPMI_PREC_BF16) return P_BF16;
    if (precision == CPMI_PREC_F32) return P_F32;
    return fail(c, CPMI_ERR_ARG, "unknown precision %d for float32 input", precision);
}

int set_device(cpmi_ctx *c)
{
    HIPCHK(c, hipSetDevice(c->device));
    return CPMI_OK;
}

// Lower bound on the distance of every pair of a tile whose blocks have the
// reference-distance intervals [loI, hiI] and [loJ, hiJ] (q references): by
// the triangle inequality |d(r,x) - d(r,y)| <= d(x,y), so the gap between the
// intervals of any one reference bounds every pair. The distances carry a
// relative rounding error far below 2^-40 (FP64 sums of at most 2^20
// squares); 2^-34 of the larger endpoint is subtracted for it.
double tile_lower_bound(const double *loI, const double *hiI, const double *loJ, const double *hiJ, int q)
{
    double lb = 0.0;
    for (int k = 0; k < q; ++k) {
        double g = std::max(loJ[k] - hiI[k], loI[k] - hiJ[k]);
        g -= 0x1p-34 * std::max(std::fabs(hiI[k]), std::fabs(hiJ[k]));
        lb = std::max(lb, g);
    }
    return lb;
}

uint64_t splitmix64(uint64_t x)
{
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// Reference-point pruning of one point set or of the windows of one series
// (Section 3, MPR steps 1-3): order the rows by their distance to the first
// projected reference (h.perm; for windows also its inverse, h.iperm, padded
// to whole 256-row blocks), or with w > 0 by buckets of width w of that
// distance and by the distance to the second reference within a bucket, and
// reduce, per block of `tile` rows in that order and per reference, the
// interval of distances (c->mlo, c->mhi: nT x q each). Queued on st only.
int prune_prepare(cpmi_ctx *c, HostProb &h, int tile, double w, hipStream_t st)
{
    const int q = c->prune_q;
    const int64_t n = h.n;
    const int64_t npad = (n + 255) / 256 * 256;
    const int dtype = h.src_i8 ? CPMI_I8 : CPMI_F32;
    const int64_t nT = (n + tile - 1) / tile;
    int rc;
    if ((rc = ensure(c, c->mD, ((size_t)q * n + (h.motif ? (size_t)q * h.d : 0)) * 8))) return rc;
    if ((rc = ensure(c, c->mperm, (size_t)npad * 4))) return rc;
    if (h.motif && (rc = ensure(c, c->miperm, (size_t)n * 4))) return rc;
    if ((rc = ensure(c, c->mlo, (size_t)nT * q * 8))) return rc;
    if ((rc = ensure(c, c->mhi, (size_t)nT * q * 8))) return rc;
    if ((rc = ensure(c, c->mrefs, (size_t)q * 4))) return rc;
    if ((rc = ensure(c, c->w.keys, (size_t)n * 8))) return rc;  // sort scratch: indices
    if ((rc = ensure(c, c->w.vals, (size_t)n * 8))) return rc;  // sorted keys
    double *D = (double *)c->mD.p;
    int32_t *perm = (int32_t *)c->mperm.p;
    const bool two = w > 0.0 && q >= 2;
    size_t tb = 0;
    if (two) HIPCHK(c, sort_ref_order2(nullptr, &tb, D, D + n, w, nullptr, nullptr, nullptr, n, st));
    else HIPCHK(c, sort_ref_order(nullptr, &tb, nullptr, nullptr, nullptr, nullptr, n, st));
    if ((rc = ensure(c, c->msort, std::max<size_t>(tb, 1)))) return rc;
    std::vector<int32_t> refs(q);
    for (int k = 0; k < q; ++k) refs[k] = (int32_t)(splitmix64(c->prune_seed * 64 + (uint64_t)k) % (uint64_t)n);
    HIPCHK(c, hipMemcpyAsync(c->mrefs.p, refs.data(), q * 4, hipMemcpyHostToDevice, st));
    if (h.motif) {
        launch_ref_dist_windows((const float *)h.src, n, h.d, (const int32_t *)c->mrefs.p, q, c->prune_f,
                                D + (size_t)q * n, D, st);
    } else {
        launch_ref_dist(h.src, dtype, n, h.d, h.ld, (const int32_t *)c->mrefs.p, q, c->prune_f, D, st);
    }
    if (two)
        HIPCHK(c, sort_ref_order2(c->msort.p, &tb, D, D + n, w, (double *)c->w.vals.p, (int32_t *)c->w.keys.p, perm,
                                  n, st));
    else
        HIPCHK(c, sort_ref_order(c->msort.p, &tb, D, (double *)c->w.vals.p, (int32_t *)c->w.keys.p, perm, n, st));
    if (h.motif) launch_perm_finish(perm, (int32_t *)c->miperm.p, n, npad, st);
    launch_block_range(D, n, q, perm, tile, nT, (double *)c->mlo.p, (double *)c->mhi.p, st);
    HIPCHK(c, hipGetLastError());
    h.perm = perm;
    if (h.motif) h.iperm = (const int32_t *)c->miperm.p;
    return CPMI_OK;
}

// Tile list of the rows in reference order without the tiles whose lower
// bound exceeds T (MPR's test of step 5, per tile). *npruned counts the
// dropped tiles. band >= 0 keeps only the tiles with J - I <= band.
void pruned_tiles(const HostProb &h, int tile, int q, const std::vector<double> &lo, const std::vector<double> &hi,
                  double T, int64_t band, std::vector<uint64_t> &tl, int64_t &nfull, int64_t &npruned)
{
    const int64_t nT = (h.n + tile - 1) / tile;
    // intervals widened by the rounding margin of tile_lower_bound, once per
    // block: [lo - m, hi + m], m = 2^-34 |hi|. A gap between widened intervals
    // subtracts mI + mJ >= 2^-34 max(|hiI|, |hiJ|), so a tile dropped here has
    // tile_lower_bound > T (the test stops at the first reference that shows
    // it)
    std::vector<double> lw((size_t)nT * q), hw((size_t)nT * q);
    for (size_t k = 0; k < lw.size(); ++k) {
        const double m = 0x1p-34 * std::fabs(hi[k]);
        lw[k] = lo[k] - m;
        hw[k] = hi[k] + m;
    }
    auto exceeds = [&](int64_t I, int64_t J) {
        if (T < 0.0) return true;
        const double *lI = &lw[I * q], *hI = &hw[I * q], *lJ = &lw[J * q], *hJ = &hw[J * q];
        for (int k = 0; k < q; ++k)
            if ((lJ[k] - hI[k] > T) | (lI[k] - hJ[k] > T)) return true;
        return false;
    };
    // the rows are ordered by reference 0 (or by buckets of it), so the least
    // widened reference-0 distance of blocks J and after, env[J], does not
    // decrease with J: jend[I] is the first block column from which on the
    // reference-0 gap alone exceeds T
    std::vector<double> env(nT);
    for (int64_t J = nT - 1; J >= 0; --J) env[J] = J + 1 < nT ? std::min(lw[J * q], env[J + 1]) : lw[J * q];
    std::vector<int64_t> jend(nT);
    for (int64_t I = 0; I < nT; ++I) {
        int64_t a = I, b = nT;
        while (a < b) {
            const int64_t m = (a + b) / 2;
            if (env[m] - hw[I * q] > T) b = m;
            else a = m + 1;
        }
        jend[I] = band >= 0 ? std::min(a, I + band + 1) : a;
    }
    std::vector<HostProb> one(1, h);
    build_tiles(
        one, tile, tl, &nfull,
        [&](int64_t I, int64_t J) { return (band < 0 || J - I <= band) && !exceeds(I, J); }, &jend);
    int64_t kept = 0;
    for (uint64_t e : tl) kept += e != TILE_NONE;
    npruned = nT * (nT + 1) / 2 - kept;
}

// Queue the device build of the pruned tile list of problem h (MPR's test of
// step 5, per tile; the intervals of the last prune_prepare) with threshold
// T_host, or sqrt(max(r2, U)) (1 + 2^-30) with U read from u_bits on the
// device, and the copy of its totals to c->plist. No synchronisation.
int queue_prune_list(cpmi_ctx *c, const HostProb &h, int tile, int q, double T_host, const unsigned long long *u_bits,
                     double r2, hipStream_t st)
{
    const int64_t nT = (h.n + tile - 1) / tile;
    const int64_t G = std::max(1, h.band);
    const int64_t S = prune_segments(nT, G);
    const bool permuted = h.motif && h.perm;
    int rc;
    if ((rc = ensure(c, c->mtl, ((size_t)nT * (nT + 1) / 2 + 8) * 8))) return rc;
    if ((rc = ensure(c, c->mseg, (size_t)S * 16))) return rc;
    if ((rc = ensure(c, c->mout4, 32))) return rc;
    size_t tb = 0;
    HIPCHK(c, launch_prune_list(nullptr, &tb, nullptr, nullptr, q, h.n, h.excl, tile, permuted, G, T_host,
                                u_bits, r2, nullptr, nullptr, nullptr, nullptr, st));
    if ((rc = ensure(c, c->mscan, std::max<size_t>(tb, 1)))) return rc;
    if (!c->plist) HIPCHK(c, hipHostMalloc((void **)&c->plist, 32, hipHostMallocDefault));
    uint64_t *seg = (uint64_t *)c->mseg.p;
    HIPCHK(c, launch_prune_list(c->mscan.p, &tb, (const double *)c->mlo.p, (const double *)c->mhi.p, q, h.n,
                                h.excl, tile, permuted, G, T_host, u_bits, r2, seg, seg + S, (uint64_t *)c->mtl.p,
                                (int64_t *)c->mout4.p, st));
    HIPCHK(c, hipMemcpyAsync(c->plist, c->mout4.p, 32, hipMemcpyDeviceToHost, st));
    return CPMI_OK;
}

// The list queued by queue_prune_list, once the stream has passed it.
DevList prune_list_of(const cpmi_ctx *c)
{
    const int64_t *o = c->plist;
    return DevList{(const uint64_t *)c->mtl.p, o[0], o[1], o[1] > 0 ? o[2] : o[3]};
}

// The exact search of one problem with reference-point tile pruning. MPR keeps
// a running upper bound of the least distance; here it comes from a first
// search over the diagonal band of the reference order (neighbouring blocks,
// where close pairs land), and the full search then skips every tile whose
// reference bound exceeds it and the radius. The full list is built on the
// device behind the band search, from the band's U as the device left it.
int pruned_search(cpmi_ctx *c, std::vector<HostProb> &hp, int prec, int tile, bool want_cpp, bool want_frnn,
                  hipStream_t st, RunOut &ro)
{
    const int q = c->prune_q;
    HostProb &h = hp[0];
    const int64_t nT = (h.n + tile - 1) / tile;
    const double r2 = want_frnn ? h.r2 : 0.0;
    // radius queries with two or more references: the two-reference order
    const bool two = want_frnn && q >= 2 && c->prune_order == 0 && r2 > 0.0 && std::isfinite(r2);
    if ((double)nT * (nT + 1.0) / 2.0 > 2147483647.0 - 1048576.0)
        return fail(c, CPMI_ERR_ARG, "problem too large for one pruned screen (%lld blocks)", (long long)nT);
    int rc;
    if ((rc = prune_prepare(c, h, tile, two ? c->prune_w * std::sqrt(r2) : 0.0, st))) return rc;
    h.band = pick_band(c, prec, h.d, (double)pairs_of(h));
    if (want_cpp) {
        // the band list needs no intervals (with T = inf no tile is dropped)
        const std::vector<double> none((size_t)nT * q, 0.0);
        std::vector<uint64_t> tl;
        int64_t nfull = 0, npruned = 0;
        pruned_tiles(h, tile, q, none, none, std::numeric_limits<double>::infinity(), 1, tl, nfull, npruned);
        // queued behind the band search: the full list from the band's U
        int frc = CPMI_OK;
        auto busy = [&]() {
            frc = queue_prune_list(c, h, tile, q, 0.0, (const unsigned long long *)c->w.res.p, r2, st);
        };
        RunOut band;
        if ((rc = run_search(c, hp, prec, tile, true, false, st, false, band, &tl, nfull, false, busy))) return rc;
        if (frc) return frc;
        if ((rc = flags_error(c, band.res[0].flags))) return rc;
    } else {
        if ((rc = queue_prune_list(c, h, tile, q, std::sqrt(r2) * (1.0 + 0x1p-30), nullptr, 0.0, st))) return rc;
        HIPCHK(c, hipStreamSynchronize(st));
    }
    const DevList dl = prune_list_of(c);
    // the band search (if any) left the screen operand in place
    if ((rc = run_search(c, hp, prec, tile, want_cpp, want_frnn, st, false, ro, nullptr, 0, want_cpp, {}, nullptr,
                         nullptr, &dl)))
        return rc;
    c->stats.tiles_pruned = nT * (nT + 1) / 2 - (c->plist[2] + c->plist[3]);
    return CPMI_OK;
}

// String problems (Sections 5 and 6): zeroed workspace for `rows` encoded
// rows of Lz int8 values, filled by `encode` (which may raise F_SYMBOL in the
// flag word), then one exact int8 closest-pair search over them. On success
// *r holds the search result (screen rows a < b and the exact squared
// distance). Synchronises.
int encoded_search(cpmi_ctx *c, HostProb &h, int64_t rows, int64_t Lz, int tile, hipStream_t st,
                   const std::function<void(signed char *, unsigned int *)> &encode, ResDev *r)
{
    int rc;
    const size_t zb = ((size_t)rows * Lz + 3) / 4 * 4;
    if ((rc = ensure(c, c->mZ, zb))) return rc;
    if ((rc = ensure(c, c->mflag, 4))) return rc;
    launch_fill_u32((uint32_t *)c->mZ.p, 0u, (int64_t)(zb / 4), st);
    launch_fill_u32((uint32_t *)c->mflag.p, 0u, 1, st);
    encode((signed char *)c->mZ.p, (unsigned int *)c->mflag.p);
    HIPCHK(c, hipGetLastError());
    unsigned int flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->mflag.p, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (flag & F_SYMBOL) return fail(c, CPMI_ERR_ARG, "a symbol lies outside the alphabet");
    h.n = rows;
    h.d = Lz;
    h.ld = Lz;
    h.excl = 1;
    h.src = c->mZ.p;
    h.src_i8 = 1;
    h.r2 = -1.0;
    std::vector<HostProb> hp(1, h);
    RunOut ro;
    if ((rc = run_search(c, hp, P_I8, tile, true, false, st, false, ro))) return rc;
    if ((rc = flags_error(c, ro.res[0].flags))) return rc;
    if (ro.res[0].best_d2 == ~0ull || ro.res[0].best_ij == ~0ull) return fail(c, CPMI_ERR_NOPAIR, "no admissible pair");
    *r = ro.res[0];
    return CPMI_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int cpmi_version(void) { return 10000; }

int cpmi_create(cpmi_ctx **out, int device, const char *tune_cache_path)
{
    if (!out) return CPMI_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return CPMI_ERR_HIP;
    if (device < 0 || device >= ndev) return CPMI_ERR_ARG;
    cpmi_ctx *c = new cpmi_ctx();
    c->device = device;
    if (hipSetDevice(device) != hipSuccess || hipEventCreate(&c->ev0) != hipSuccess ||
        hipEventCreate(&c->ev1) != hipSuccess || hipEventCreate(&c->es0) != hipSuccess ||
        hipEventCreate(&c->es1) != hipSuccess ||
        hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return CPMI_ERR_HIP;
    }
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        c->ncu = ncu;
    if (device < kMaxDevices) {
        // the static scratch's address on this device, taken once per device
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_addr[device]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
                hipEventDestroy(c->ev0);
                hipEventDestroy(c->ev1);
                hipEventDestroy(c->es0);
                hipEventDestroy(c->es1);
                hipStreamDestroy(c->own);
                delete c;
                return CPMI_ERR_HIP;
            }
            g_scratch_addr[device] = p;
        }
        c->scratch = g_scratch_addr[device];
    }
    load_tune_cache(c, tune_cache_path);
    *out = c;
    return CPMI_OK;
}

int cpmi_destroy(cpmi_ctx *c)
{
    if (!c) return CPMI_OK;
    hipSetDevice(c->device);
    hipDeviceSynchronize();
    if (c->gexec) hipGraphExecDestroy(c->gexec);
    DevBuf *bufs[] = {&c->w.xs,      &c->w.shat,  &c->w.bmax, &c->w.musg, &c->w.probs, &c->w.jobs, &c->w.tiles, &c->w.tile_min,
                      &c->w.sel,     &c->w.candR, &c->w.candU, &c->w.cand_d2, &c->w.keys, &c->w.vals, &c->w.cnt, &c->w.ubits,
                      &c->w.res,     &c->mD,    &c->mperm, &c->miperm, &c->mlo, &c->mhi, &c->mrefs, &c->msort, &c->w.mrowstat,
                      &c->mZ,      &c->mflag, &c->lbA, &c->lbT, &c->lbC, &c->lbP, &c->lbK, &c->mtl, &c->mseg,
                      &c->mscan,   &c->mout4, &c->csrW, &c->csrT, &c->srtK, &c->srtV, &c->srtT};
    for (DevBuf *b : bufs)
        if (b->p) hipFree(b->p);
    if (c->pinned) hipHostFree(c->pinned);
    if (c->plist) hipHostFree(c->plist);
    if (c->ev0) hipEventDestroy(c->ev0);
    if (c->ev1) hipEventDestroy(c->ev1);
    if (c->es0) hipEventDestroy(c->es0);
    if (c->es1) hipEventDestroy(c->es1);
    if (c->own) hipStreamDestroy(c->own);
    delete c;
    return CPMI_OK;
}

const char *cpmi_last_error(cpmi_ctx *c) { return c ? c->err.c_str() : "null context"; }

int cpmi_pairs_to_csr(cpmi_ctx *c, const int64_t *pairs, int64_t m, int64_t n, int64_t *row_ptr, int64_t *cols,
                      void *stream)
{
    if (!c) return CPMI_ERR_ARG;
    if (n < 1 || n >= ((int64_t)1 << 31) || m < 0 || m >= ((int64_t)1 << 31) || !row_ptr ||
        (m > 0 && (!pairs || !cols)))
        return fail(c, CPMI_ERR_ARG, "pairs_to_csr: bad arguments (n %lld, m %lld)", (long long)n, (long long)m);
    hipSetDevice(c->device);
    const hipStream_t st = (hipStream_t)stream;
    size_t sort_bytes = 0;
    const size_t wb = csr_scratch_bytes(m, n, &sort_bytes);
    int rc;
    if ((rc = ensure(c, c->csrW, wb))) return rc;
    if ((rc = ensure(c, c->csrT, sort_bytes))) return rc;
    unsigned int *bad = (unsigned int *)((char *)c->csrW.p + (wb - 256));
    HIPCHK(c, launch_pairs_to_csr(pairs, m, n, row_ptr, cols, c->csrW.p, c->csrT.p, sort_bytes, bad, st));
    if ((rc = ensure_pinned(c, 4))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->pinned, bad, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    if (*(unsigned int *)c->pinned)
        return fail(c, CPMI_ERR_ARG, "pairs_to_csr: a pair outside 0 <= i < j < %lld", (long long)n);
    return CPMI_OK;
}

int cpmi_last_stats(cpmi_ctx *c, cpmi_stats *out)
{
    if (!c || !out) return CPMI_ERR_ARG;
    *out = c->stats;
    return CPMI_OK;
}

int cpmi_set_pruning(cpmi_ctx *c, int q, double f, uint64_t seed)
{
    if (!c) return CPMI_ERR_ARG;
    if (q < 0 || q > 32) return fail(c, CPMI_ERR_ARG, "q must be in 0..32");
    if (!(f > 0.0) || !std::isfinite(f)) return fail(c, CPMI_ERR_ARG, "f must be finite and > 0");
    c->prune_q = q;
    c->prune_f = f;
    c->prune_seed = seed;
    return CPMI_OK;
}

int cpmi_set_tile(cpmi_ctx *c, int precision, int tile)
{
    if (!c || precision < 1 || precision > 3) return CPMI_ERR_ARG;
    if (tile != 0 && tile != 128 && tile != 256) return fail(c, CPMI_ERR_ARG, "tile must be 0, 128 or 256");
    c->tile_override[precision] = tile;
    return CPMI_OK;
}

int cpmi_points(cpmi_ctx *c, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, int precision, double R2,
                void *stream, cpmi_pair *best, int64_t *pairs, double *d2, int64_t cap, int64_t *count_out)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    const bool want_frnn = R2 >= 0.0;
    const bool want_cpp = best != nullptr;
    if (best) memset(best, 0, sizeof *best);
    if (count_out) *count_out = 0;
    if (!pts) return fail(c, CPMI_ERR_ARG, "points pointer is NULL");
    if (dtype != CPMI_F32 && dtype != CPMI_I8) return fail(c, CPMI_ERR_ARG, "unknown dtype %d", dtype);
    if (d < 1 || ld < d || n < 0) return fail(c, CPMI_ERR_ARG, "bad shape n=%lld d=%lld ld=%lld", (long long)n, (long long)d, (long long)ld);
    if (n >= (1ll << 31) - 256) return fail(c, CPMI_ERR_ARG, "n must be below 2^31");
    if (dtype == CPMI_I8 && d > 32768) return fail(c, CPMI_ERR_ARG, "int8 dimension must be <= 32768 (int32 Gram)");
    if (d > (1 << 20)) return fail(c, CPMI_ERR_ARG, "dimension must be <= 2^20");
    if (!want_cpp && !want_frnn) return fail(c, CPMI_ERR_ARG, "nothing requested (best == NULL and R2 < 0)");
    if (want_frnn && ((cap > 0 && !pairs) || !count_out || cap < 0))
        return fail(c, CPMI_ERR_ARG, "radius search needs count_out, cap >= 0 and pairs (unless cap == 0)");
    if (std::isnan(R2)) return fail(c, CPMI_ERR_ARG, "R2 is NaN");
    if (n < 2) {
        if (best) best->status = CPMI_ERR_NOPAIR, best->i = best->j = -1;
        return fail(c, CPMI_ERR_NOPAIR, "fewer than two points");
    }
    const double npairs = (double)pairs_of(n, 1);
    const int prec = resolve_prec(c, dtype, precision, d, npairs);
    if (prec < 0) return prec;
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::vector<HostProb> hp(1);
    hp[0].n = n;
    hp[0].d = d;
    hp[0].ld = ld;
    hp[0].excl = 1;
    hp[0].src = pts;
    hp[0].src_i8 = dtype == CPMI_I8;
    hp[0].r2 = want_frnn ? R2 : -1.0;
    const int tile = pick_tile(c, prec, d, npairs);
    RunOut ro;
    if (c->prune_q > 0 && n > tile) {
        if ((rc = pruned_search(c, hp, prec, tile, want_cpp, want_frnn, st, ro))) return rc;
    } else {
        if ((rc = run_search(c, hp, prec, tile, want_cpp, want_frnn, st, false, ro))) return rc;
    }
    if ((rc = flags_error(c, ro.res[0].flags))) return rc;
    if (want_cpp) {
        fill_pair(ro.res[0], best);
        if (best->status) return fail(c, best->status, "no admissible pair");
    }
    if (want_frnn) return finish_frnn(c, ro, st, pairs, d2, cap, count_out);
    return CPMI_OK;
}

int cpmi_closest_pair(cpmi_ctx *c, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, int precision,
                      void *stream, cpmi_pair *out)
{
    if (!out) return c ? fail(c, CPMI_ERR_ARG, "out is NULL") : CPMI_ERR_ARG;
    return cpmi_points(c, pts, dtype, n, d, ld, precision, -1.0, stream, out, nullptr, nullptr, 0, nullptr);
}

int cpmi_closest_pair_noalloc(cpmi_ctx *c, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld,
                              int precision, void *stream, cpmi_pair *out)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    if (!out) return fail(c, CPMI_ERR_ARG, "out is NULL");
    memset(out, 0, sizeof *out);
    out->i = out->j = -1;
    if (!pts) return fail(c, CPMI_ERR_ARG, "points pointer is NULL");
    if (dtype != CPMI_F32 && dtype != CPMI_I8) return fail(c, CPMI_ERR_ARG, "unknown dtype %d", dtype);
    if (d < 1 || ld < d || n < 0)
        return fail(c, CPMI_ERR_ARG, "bad shape n=%lld d=%lld ld=%lld", (long long)n, (long long)d, (long long)ld);
    if (dtype == CPMI_I8 && d > 32768) return fail(c, CPMI_ERR_ARG, "int8 dimension must be <= 32768 (int32 Gram)");
    if (!c->scratch) return fail(c, CPMI_ERR_ARG, "no static scratch on device %d", c->device);
    if (n < 2) {
        out->status = CPMI_ERR_NOPAIR;
        return fail(c, CPMI_ERR_NOPAIR, "fewer than two points");
    }
    const double npairs = (double)pairs_of(n, 1);
    const int prec = resolve_prec(c, dtype, precision, d, npairs);
    if (prec < 0) return prec;
    const int tile = pick_tile(c, prec, d, npairs);
    // reject what cannot fit before any work is queued: the screen operand
    // and row scalars alone
    const int64_t npad = (n + 255) / 256 * 256;
    const double need = (double)npad * kpad_for(prec, d, tile) * elem_bytes(prec) + (double)npad * 4.0;
    if (need > (double)kScratchBytes)
        return fail(c, CPMI_ERR_CAPACITY, "%lld x %lld points need %.0f bytes of screen operand; the static scratch "
                    "holds %zu", (long long)n, (long long)d, need, kScratchBytes);
    int rc;
    if ((rc = set_device(c))) return rc;
    std::vector<HostProb> hp(1);
    hp[0].n = n;
    hp[0].d = d;
    hp[0].ld = ld;
    hp[0].excl = 1;
    hp[0].src = pts;
    hp[0].src_i8 = dtype == CPMI_I8;
    hp[0].r2 = -1.0;
    Arena ar;
    ar.base = (char *)c->scratch;
    ar.size = kScratchBytes;
    RunOut ro;
    if ((rc = run_search(c, hp, prec, tile, true, false, (hipStream_t)stream, false, ro, nullptr, 0, false, {}, &ar)))
        return rc;
    if ((rc = flags_error(c, ro.res[0].flags))) return rc;
    fill_pair(ro.res[0], out);
    if (out->status) return fail(c, out->status, "no admissible pair");
    return CPMI_OK;
}

int cpmi_frnn(cpmi_ctx *c, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, double R2, int precision,
              void *stream, int64_t *pairs, double *d2, int64_t cap, int64_t *count_out)
{
    if (!(R2 >= 0.0)) return c ? fail(c, CPMI_ERR_ARG, "R2 must be >= 0") : CPMI_ERR_ARG;
    if (c && n < 2 && n >= 0 && d >= 1 && ld >= d && pts) {
        if (count_out) *count_out = 0;
        return CPMI_OK;  // no pair can be within the radius
    }
    return cpmi_points(c, pts, dtype, n, d, ld, precision, R2, stream, nullptr, pairs, d2, cap, count_out);
}

int cpmi_motif(cpmi_ctx *c, const float *series, int64_t len, int64_t ell, int64_t excl, int precision, double R2,
               void *stream, cpmi_pair *best, int64_t *pairs, double *d2, int64_t cap, int64_t *count_out)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    const bool want_frnn = R2 >= 0.0;
    const bool want_cpp = best != nullptr;
    if (best) memset(best, 0, sizeof *best);
    if (count_out) *count_out = 0;
    if (!series) return fail(c, CPMI_ERR_ARG, "series pointer is NULL");
    if (ell < 2 || len < ell) return fail(c, CPMI_ERR_ARG, "need 2 <= ell <= len (ell=%lld len=%lld)", (long long)ell, (long long)len);
    if (ell > SERIES_MAX_ELL) return fail(c, CPMI_ERR_ARG, "ell must be <= %d", SERIES_MAX_ELL);
    if (len >= (1ll << 31) - 256) return fail(c, CPMI_ERR_ARG, "len must be below 2^31");
    if (!want_cpp && !want_frnn) return fail(c, CPMI_ERR_ARG, "nothing requested (best == NULL and R2 < 0)");
    if (want_frnn && ((cap > 0 && !pairs) || !count_out || cap < 0))
        return fail(c, CPMI_ERR_ARG, "radius search needs count_out, cap >= 0 and pairs (unless cap == 0)");
    if (std::isnan(R2)) return fail(c, CPMI_ERR_ARG, "R2 is NaN");
    if (precision != CPMI_PREC_AUTO && precision != CPMI_PREC_F32 && precision != CPMI_PREC_BF16)
        return fail(c, CPMI_ERR_ARG, "motif precision must be AUTO, F32 or BF16");
    if (excl <= 0) excl = ell;
    const int64_t N = len - ell + 1;
    if (N <= excl) {
        if (best) best->status = CPMI_ERR_NOPAIR, best->i = best->j = -1;
        return fail(c, CPMI_ERR_NOPAIR, "no admissible window pair (windows=%lld, exclusion=%lld)", (long long)N, (long long)excl);
    }
    const double npairs = (double)pairs_of(N, excl);
    const int prec = resolve_prec(c, CPMI_F32, precision, ell, npairs);
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::vector<HostProb> hp(1);
    hp[0].n = N;
    hp[0].d = ell;
    hp[0].ld = 1;
    hp[0].excl = excl;
    hp[0].motif = 1;
    hp[0].src = series;
    hp[0].len = len;
    hp[0].r2 = want_frnn ? R2 : -1.0;
    RunOut ro;
    if (c->prune_q > 0 && N > 256 && excl <= (1 << 30)) {
        // windows in reference order: only the 256-row screen applies the
        // exclusion zone to permuted rows (in 32-bit unsigned arithmetic,
        // hence the bound on excl)
        if ((rc = pruned_search(c, hp, prec, 256, want_cpp, want_frnn, st, ro))) return rc;
    } else {
        const int tile = pick_tile(c, prec, ell, npairs);
        if ((rc = run_search(c, hp, prec, tile, want_cpp, want_frnn, st, false, ro))) return rc;
    }
    if ((rc = flags_error(c, ro.res[0].flags))) return rc;
    if (want_cpp) {
        fill_pair(ro.res[0], best);
        if (best->status) return fail(c, best->status, "no admissible pair");
    }
    if (want_frnn) return finish_frnn(c, ro, st, pairs, d2, cap, count_out);
    return CPMI_OK;
}

int cpmi_motif_batch(cpmi_ctx *c, const float *const *series, const int64_t *lens, const int64_t *ells,
                     int64_t nseries, int precision, void *stream, cpmi_pair *best)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    if (!series || !lens || !ells || !best || nseries < 1) return fail(c, CPMI_ERR_ARG, "bad batch arguments");
    if (nseries > (1 << 20)) return fail(c, CPMI_ERR_ARG, "at most 2^20 series per batch");
    if (precision != CPMI_PREC_AUTO && precision != CPMI_PREC_F32 && precision != CPMI_PREC_BF16)
        return fail(c, CPMI_ERR_ARG, "motif precision must be AUTO, F32 or BF16");
    std::vector<HostProb> hp;
    std::vector<int64_t> idx;  // batch position of each problem
    int64_t ellmax = 0;
    double npairs = 0.0;
    for (int64_t s = 0; s < nseries; ++s) {
        memset(&best[s], 0, sizeof best[s]);
        best[s].i = best[s].j = -1;
        const int64_t L = lens[s], ell = ells[s];
        if (!series[s] || ell < 2 || ell > SERIES_MAX_ELL || L < ell || L >= (1ll << 31) - 256)
            return fail(c, CPMI_ERR_ARG, "series %lld: bad arguments (len=%lld ell=%lld)", (long long)s, (long long)L, (long long)ell);
        const int64_t N = L - ell + 1;
        if (N <= ell) {
            best[s].status = CPMI_ERR_NOPAIR;
            continue;
        }
        HostProb h;
        h.n = N;
        h.d = ell;
        h.ld = 1;
        h.excl = ell;
        h.motif = 1;
        h.src = series[s];
        h.len = L;
        hp.push_back(h);
        idx.push_back(s);
        ellmax = std::max<int64_t>(ellmax, ell);
        npairs += (double)pairs_of(N, ell);
    }
    if (hp.empty()) return CPMI_OK;
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (!st) {
        // graphs cannot be captured on the null stream: run on the context's
        // own stream, ordered after the work already queued on the null stream
        HIPCHK(c, hipEventRecord(c->ev0, nullptr));
        HIPCHK(c, hipStreamWaitEvent(c->own, c->ev0, 0));
        st = c->own;
    }
    const int prec = resolve_prec(c, CPMI_F32, precision, ellmax, npairs);
    const int tile = pick_tile(c, prec, ellmax, npairs);
    RunOut ro;
    if ((rc = run_search(c, hp, prec, tile, true, false, st, true, ro))) return rc;
    for (size_t p = 0; p < hp.size(); ++p) {
        cpmi_pair &b = best[idx[p]];
        const int fe = flags_error(c, ro.res[p].flags);
        if (fe) {
            b.status = fe;
            continue;
        }
        fill_pair(ro.res[p], &b);
    }
    c->err.clear();
    return CPMI_OK;
}

int cpmi_strings_pair(cpmi_ctx *c, const int8_t *strings, int64_t n, int64_t k, int64_t ld, int sigma, int mode,
                      void *stream, cpmi_match_pair *out)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    if (!out) return fail(c, CPMI_ERR_ARG, "out is NULL");
    memset(out, 0, sizeof *out);
    out->i = out->j = -1;
    if (!strings) return fail(c, CPMI_ERR_ARG, "strings pointer is NULL");
    if (mode != CPMI_MOST_CORRELATED && mode != CPMI_LEAST_CORRELATED) return fail(c, CPMI_ERR_ARG, "unknown mode %d", mode);
    if (sigma < 2 || sigma > 64) return fail(c, CPMI_ERR_ARG, "sigma must be in 2..64");
    if (k < 1 || ld < k || n < 0) return fail(c, CPMI_ERR_ARG, "bad shape n=%lld k=%lld ld=%lld", (long long)n, (long long)k, (long long)ld);
    if ((int64_t)sigma * k > (1 << 20)) return fail(c, CPMI_ERR_ARG, "sigma * k must be <= 2^20");
    if (n >= (1ll << 30)) return fail(c, CPMI_ERR_ARG, "n must be below 2^30");
    if (n < 2) {
        out->status = CPMI_ERR_NOPAIR;
        return fail(c, CPMI_ERR_NOPAIR, "fewer than two strings");
    }
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t Lz = (int64_t)sigma * k;
    const bool least = mode == CPMI_LEAST_CORRELATED;
    HostProb h;
    int64_t rows = n;
    int tile;
    if (least) {
        // codes in rows [0, n), complements from the next multiple of 256
        h.split = (n + 255) / 256 * 256;
        h.na = n;
        rows = h.split + n;
        tile = 256;
    } else {
        tile = pick_tile(c, P_I8, Lz, (double)pairs_of(n, 1));
    }
    ResDev r;
    if ((rc = encoded_search(c, h, rows, Lz, tile, st,
                             [&](signed char *Z, unsigned int *flag) {
                                 launch_encode_strings((const signed char *)strings, n, k, ld, sigma, least ? 1 : 0, Z,
                                                       Lz, h.split, flag, st);
                             },
                             &r)))
        return rc;
    const int64_t a = (int64_t)(r.best_ij >> 32), b = (int64_t)(r.best_ij & 0xffffffffu);
    const int64_t d2 = (int64_t)__builtin_bit_cast(double, (uint64_t)r.best_d2);
    out->i = a;
    out->j = least ? b - h.split : b;
    // code vs code: d2 = 2 (k - u); code vs complement: d2 = sigma k - 2 (k - u)
    out->matches = least ? k - (Lz - d2) / 2 : k - d2 / 2;
    out->length = k;
    out->status = CPMI_OK;
    c->stats.valid_pairs = pairs_of(n, 1);
    return CPMI_OK;
}

int cpmi_strings_lightbulb(cpmi_ctx *c, const int8_t *strings, int64_t n, int64_t k, int64_t ld, int sigma,
                           int mode, int iterations, int columns, uint64_t seed, int64_t cap, void *stream,
                           cpmi_match_pair *out, int64_t *pairs_out)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    if (!out) return fail(c, CPMI_ERR_ARG, "out is NULL");
    memset(out, 0, sizeof *out);
    out->i = out->j = -1;
    if (pairs_out) *pairs_out = 0;
    if (!strings) return fail(c, CPMI_ERR_ARG, "strings pointer is NULL");
    if (mode != CPMI_MOST_CORRELATED && mode != CPMI_LEAST_CORRELATED) return fail(c, CPMI_ERR_ARG, "unknown mode %d", mode);
    if (sigma < 2 || sigma > 64) return fail(c, CPMI_ERR_ARG, "sigma must be in 2..64");
    if (k < 1 || ld < k || n < 0) return fail(c, CPMI_ERR_ARG, "bad shape n=%lld k=%lld ld=%lld", (long long)n, (long long)k, (long long)ld);
    if (n >= (1ll << 21) - 1) return fail(c, CPMI_ERR_ARG, "n must be below 2^21 - 1");
    // the best pair is packed as count << 42 | pair, the count (at most k) in 22 bits
    if (k >= (1ll << 22)) return fail(c, CPMI_ERR_ARG, "k must be below 2^22");
    if (iterations < 1) return fail(c, CPMI_ERR_ARG, "iterations must be >= 1");
    if (cap < 1 || cap > (1ll << 30)) return fail(c, CPMI_ERR_ARG, "cap must be in 1..2^30");
    int bits_per = 1;
    while ((1 << bits_per) < sigma) ++bits_per;
    if (mode == CPMI_LEAST_CORRELATED) bits_per = 1;
    const int64_t ncol_all = mode == CPMI_MOST_CORRELATED ? k : (int64_t)sigma * k;
    if (columns < 1 || columns > ncol_all || (int64_t)columns * bits_per > 64)
        return fail(c, CPMI_ERR_ARG, "columns must be in 1..min(%lld, %d)", (long long)ncol_all, 64 / bits_per);
    if (n < 2) {
        out->status = CPMI_ERR_NOPAIR;
        return fail(c, CPMI_ERR_NOPAIR, "fewer than two strings");
    }
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int m = mode == CPMI_MOST_CORRELATED ? 0 : 1;
    const int64_t total = m == 0 ? n : 2 * n;
    // columns of every iteration, distinct within an iteration (seeded
    // partial Fisher-Yates draws)
    std::vector<int32_t> cols((size_t)iterations * columns);
    {
        std::vector<int32_t> pool((size_t)ncol_all);
        uint64_t ctr = seed * 0x9e3779b97f4a7c15ull;
        for (int it = 0; it < iterations; ++it) {
            for (int64_t q = 0; q < ncol_all; ++q) pool[q] = (int32_t)q;
            for (int q = 0; q < columns; ++q) {
                const int64_t r = q + (int64_t)(splitmix64(ctr++) % (uint64_t)(ncol_all - q));
                std::swap(pool[q], pool[r]);
                cols[(size_t)it * columns + q] = pool[q];
            }
        }
    }
    // iterations in batches of B <= 256 (keys, rows, their sorted copies and
    // the pair counts and offsets of a batch within 160 MiB)
    const int B = (int)std::min<int64_t>(std::min(iterations, 256),
                                         std::max<int64_t>(1, ((int64_t)160 << 20) / (total * 40)));
    const int key_bits = columns * bits_per;
    std::vector<int32_t> seg((size_t)B + 1);
    for (int b = 0; b <= B; ++b) seg[b] = (int32_t)(b * total);
    size_t tb = 0;
    {
        // scratch of the sort: the largest of the full and the last batch
        const int Bl = iterations % B ? iterations % B : B;
        size_t t1 = 0, t2 = 0;
        HIPCHK(c, lb_sort(nullptr, &t1, nullptr, nullptr, nullptr, nullptr, total, B, nullptr, key_bits, st));
        HIPCHK(c, lb_sort(nullptr, &t2, nullptr, nullptr, nullptr, nullptr, total, Bl, nullptr, key_bits, st));
        tb = std::max(std::max(t1, t2), lb_scan_bytes((int64_t)B * total));
    }
    // keys in, keys out, rows in, rows out, pairs per position, their prefix sums
    if ((rc = ensure(c, c->lbA, (size_t)B * total * 40))) return rc;
    if ((rc = ensure(c, c->lbT, std::max<size_t>(tb, 1)))) return rc;
    if ((rc = ensure(c, c->lbC, (cols.size() + seg.size()) * 4))) return rc;
    if ((rc = ensure(c, c->lbK, 16 + (size_t)B * 16))) return rc;
    uint64_t *kin = (uint64_t *)c->lbA.p, *kout = kin + (size_t)B * total;
    int32_t *rin = (int32_t *)(kout + (size_t)B * total), *rout = rin + (size_t)B * total;
    uint64_t *num = (uint64_t *)(rout + (size_t)B * total), *poff = num + (size_t)B * total;
    const int32_t *dcols = (const int32_t *)c->lbC.p, *dseg = dcols + cols.size();
    // lbK: best pair, symbol flag, then the pairs of each iteration of a batch
    unsigned long long *best = (unsigned long long *)c->lbK.p;
    unsigned int *flag = (unsigned int *)(best + 1);
    uint64_t *segcnt = (uint64_t *)(best + 2);
    {
        std::vector<int32_t> up(cols);
        up.insert(up.end(), seg.begin(), seg.end());
        HIPCHK(c, hipMemcpyAsync(c->lbC.p, up.data(), up.size() * 4, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));   // `up` is released below
    }
    launch_fill_u64((uint64_t *)best, m == 0 ? 0ull : ~0ull, 1, st);
    launch_fill_u32(flag, 0u, 2, st);
    launch_check_symbols((const signed char *)strings, n, k, ld, sigma, flag, st);
    uint64_t collected = 0;
    std::vector<uint64_t> hc((size_t)B + 2), ho((size_t)B);
    // candidates of one fill within max(cap, 2^26) pairs (each iteration's are
    // at most cap once counted)
    const uint64_t fill_max = std::max<uint64_t>((uint64_t)cap, (uint64_t)1 << 26);
    for (int it0 = 0; it0 < iterations; it0 += B) {
        const int nb = std::min(B, iterations - it0);
        launch_lb_keys((const signed char *)strings, n, ld, sigma, m, bits_per, dcols + (size_t)it0 * columns, columns,
                       nb, kin, rin, st);
        HIPCHK(c, lb_sort(c->lbT.p, &tb, kin, kout, rin, rout, total, nb, dseg, key_bits, st));
        // pairs per sorted position, their offsets, the pairs of each iteration
        launch_lb_count(kout, rout, total, nb, n, m, num, poff, c->lbT.p, c->lbT.cap, segcnt, st);
        // (best and the symbol flag come along: a bad symbol is reported first)
        HIPCHK(c, hipMemcpyAsync(hc.data(), best, 16 + (size_t)nb * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        if ((uint32_t)hc[1] & F_SYMBOL) return fail(c, CPMI_ERR_ARG, "a symbol lies outside the alphabet");
        bool over = false;
        for (int b = 0; b < nb; ++b) {
            const uint64_t v = hc[2 + b];
            collected += v;
            over |= v > (uint64_t)cap;
            ho[b] = b ? ho[b - 1] + hc[2 + b - 1] : 0;   // first pair of iteration b in the batch
        }
        if (over) {
            if (pairs_out) *pairs_out = (int64_t)collected;
            return fail(c, CPMI_ERR_CAPACITY, "a bucketing pass produced more than %lld candidate pairs; "
                                              "choose more columns or a larger cap", (long long)cap);
        }
        // write and verify the candidates of consecutive iterations, as many
        // as one fill holds (groups [b0, b1) found first, so that the buffer
        // is sized before any fill is queued)
        std::vector<std::pair<int, int>> groups;
        uint64_t most = 0;
        for (int b0 = 0; b0 < nb;) {
            uint64_t msum = hc[2 + b0];
            int b1 = b0 + 1;
            while (b1 < nb && msum + hc[2 + b1] <= fill_max) msum += hc[2 + b1++];
            groups.emplace_back(b0, b1);
            most = std::max(most, msum);
            b0 = b1;
        }
        if (most == 0) continue;
        if ((rc = ensure(c, c->lbP, (size_t)most * 8))) return rc;
        for (auto [b0, b1] : groups) {
            const uint64_t msum = (b1 < nb ? ho[b1] : ho[nb - 1] + hc[2 + nb - 1]) - ho[b0];
            if (msum == 0) continue;
            launch_lb_fill(kout, rout, total, (int64_t)b0 * total, (int64_t)b1 * total, n, m, poff, ho[b0],
                           (int2 *)c->lbP.p, st);
            launch_lb_verify((const signed char *)strings, k, ld, m, (const int2 *)c->lbP.p, msum, best, st);
        }
    }
    HIPCHK(c, hipGetLastError());
    uint64_t res[2];
    HIPCHK(c, hipMemcpyAsync(res, c->lbK.p, 16, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    const uint32_t flag_h = (uint32_t)res[1];
    if (flag_h & F_SYMBOL) return fail(c, CPMI_ERR_ARG, "a symbol lies outside the alphabet");
    if (pairs_out) *pairs_out = (int64_t)collected;
    const uint64_t b = res[0];
    if ((m == 0 && b == 0) || (m == 1 && b == ~0ull)) {
        out->status = CPMI_ERR_NOPAIR;
        return fail(c, CPMI_ERR_NOPAIR, "no pair shared a bucket");
    }
    const uint64_t mask = (1ull << 42) - 1, ij = m == 0 ? (~b & mask) : (b & mask);
    out->i = (int64_t)(ij >> 21);
    out->j = (int64_t)(ij & ((1ull << 21) - 1));
    out->matches = (int64_t)(b >> 42);
    out->length = k;
    out->status = CPMI_OK;
    c->stats.valid_pairs = pairs_of(n, 1);
    return CPMI_OK;
}

int cpmi_two_locus(cpmi_ctx *c, const int8_t *genotypes, int64_t m1, int64_t m2, int64_t n, int64_t ld,
                   int direction, void *stream, cpmi_match_pair *out)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    c->stats = cpmi_stats{};
    if (!out) return fail(c, CPMI_ERR_ARG, "out is NULL");
    memset(out, 0, sizeof *out);
    out->i = out->j = -1;
    if (!genotypes) return fail(c, CPMI_ERR_ARG, "genotypes pointer is NULL");
    if (direction != 0 && direction != 1) return fail(c, CPMI_ERR_ARG, "direction must be 0 or 1");
    if (m1 < 1 || m2 < 1 || n < 0 || ld < n) return fail(c, CPMI_ERR_ARG, "bad shape m1=%lld m2=%lld n=%lld ld=%lld", (long long)m1, (long long)m2, (long long)n, (long long)ld);
    if (3 * (m1 + m2) > (1 << 20)) return fail(c, CPMI_ERR_ARG, "3 (m1 + m2) must be <= 2^20");
    if (n >= (1ll << 30)) return fail(c, CPMI_ERR_ARG, "n must be below 2^30");
    if (n < 2) {
        out->status = CPMI_ERR_NOPAIR;
        return fail(c, CPMI_ERR_NOPAIR, "fewer than two SNPs");
    }
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t Lz = 3 * (m1 + m2);
    HostProb h;
    h.split = (n + 255) / 256 * 256;
    h.na = n;
    ResDev r;
    if ((rc = encoded_search(c, h, h.split + n, Lz, 256, st,
                             [&](signed char *Z, unsigned int *flag) {
                                 launch_encode_two_locus((const signed char *)genotypes, m1, m2, n, ld, direction, Z,
                                                         Lz, h.split, flag, st);
                             },
                             &r)))
        return rc;
    const int64_t a = (int64_t)(r.best_ij >> 32), b = (int64_t)(r.best_ij & 0xffffffffu);
    const int64_t d2 = (int64_t)__builtin_bit_cast(double, (uint64_t)r.best_d2);
    out->i = a;
    out->j = b - h.split;
    out->matches = Lz - d2;   // 0/1 rows: squared distance = mismatching bits
    out->length = Lz;
    out->status = CPMI_OK;
    c->stats.valid_pairs = pairs_of(n, 1);
    return CPMI_OK;
}

int cpmi_autotune(cpmi_ctx *c, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, int precision,
                  void *stream, int reps, cpmi_tune_result *out)
{
    if (!c) return CPMI_ERR_ARG;
    if (!out || reps < 1 || reps > 1000) return fail(c, CPMI_ERR_ARG, "autotune needs out and 1 <= reps <= 1000");
    memset(out, 0, sizeof *out);
    if (n < 2 || d < 1 || ld < d || !pts) return fail(c, CPMI_ERR_ARG, "autotune needs n >= 2 points");
    std::vector<int> precs;
    if (dtype == CPMI_I8) {
        if (precision != CPMI_PREC_AUTO && precision != CPMI_PREC_I8)
            return fail(c, CPMI_ERR_ARG, "int8 points take CPMI_PREC_I8 (or AUTO)");
        precs.push_back(P_I8);
    } else if (dtype == CPMI_F32) {
        if (precision == CPMI_PREC_AUTO) precs = {P_F32, P_BF16};
        else if (precision == CPMI_PREC_F32 || precision == CPMI_PREC_BF16) precs.push_back(precision);
        else return fail(c, CPMI_ERR_ARG, "unknown precision %d for float32 input", precision);
    } else {
        return fail(c, CPMI_ERR_ARG, "unknown dtype %d", dtype);
    }
    const int kb = kbucket(d), rb = rbucket((double)pairs_of(n, 1));
    const int tiles[2] = {128, 256};
    int band_of[4] = {0, 0, 0, 0};
    double best_all = 0.0;
    for (int p : precs) {
        const int saved = c->tile_override[p];
        double best = 0.0;
        int best_tile = 0;
        for (int ti = 0; ti < 2; ++ti) {
            c->tile_override[p] = tiles[ti];
            double tmin = 0.0;
            for (int r = 0; r <= reps; ++r) {  // the first call warms up
                cpmi_pair bp;
                const int rc = cpmi_points(c, pts, dtype, n, d, ld, p, -1.0, stream, &bp, nullptr, nullptr, 0,
                                           nullptr);
                if (rc) {
                    c->tile_override[p] = saved;
                    return rc;
                }
                if (r > 0 && (tmin == 0.0 || c->stats.kernel_ms < tmin)) tmin = c->stats.kernel_ms;
            }
            out->ms[p][ti] = tmin;
            if (best_tile == 0 || tmin < best) best = tmin, best_tile = tiles[ti];
        }
        c->tile_override[p] = saved;
        set_tuned(c, p, kb, rb, best_tile);
        if (best_tile == 256) {
            // the band height of the tile order (block rows per band): panel
            // reuse in L2 against the spread of the work-groups of one XCD
            const int bands[3] = {4, 8, 16};
            c->tile_override[p] = 256;
            double bbest = 0.0;
            int bb = BAND_DEFAULT;
            for (int bi = 0; bi < 3; ++bi) {
                c->band_override = bands[bi];
                double tmin = 0.0;
                for (int r = 0; r <= reps; ++r) {
                    cpmi_pair bp;
                    const int rc = cpmi_points(c, pts, dtype, n, d, ld, p, -1.0, stream, &bp, nullptr, nullptr, 0,
                                               nullptr);
                    if (rc) {
                        c->tile_override[p] = saved;
                        c->band_override = 0;
                        return rc;
                    }
                    if (r > 0 && (tmin == 0.0 || c->stats.kernel_ms < tmin)) tmin = c->stats.kernel_ms;
                }
                out->band_ms[p][bi] = tmin;
                if (bi == 0 || tmin < bbest) bbest = tmin, bb = bands[bi];
            }
            c->band_override = 0;
            c->tile_override[p] = saved;
            set_tuned(c, p, kb, rb, bb, KIND_BAND);
            band_of[p] = bb;
        }
        if (out->precision == 0 || best < best_all) {
            best_all = best;
            out->precision = p;
            out->tile = best_tile;
        }
    }
    if (precs.size() > 1) set_tuned(c, 0, kb, rb, out->precision);
    out->band = band_of[out->precision];
    c->err.clear();
    return CPMI_OK;
}

int cpmi_save_tune_cache(cpmi_ctx *c, const char *path)
{
    if (!c) return CPMI_ERR_ARG;
    if (!path) return fail(c, CPMI_ERR_ARG, "path is NULL");
    std::vector<TuneEntry> t = c->tuned;
    std::sort(t.begin(), t.end(), [](const TuneEntry &a, const TuneEntry &b) {
        return std::make_tuple(a.kind, a.prec, a.kb, a.rb) < std::make_tuple(b.kind, b.prec, b.kb, b.rb);
    });
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(c, CPMI_ERR_ARG, "cannot write %s", tmp.c_str());
    fprintf(f, "{");
    for (size_t k = 0; k < t.size(); ++k)
        fprintf(f, "%s\n \"%s%s:k%d:r%d\": %d", k ? "," : "", t[k].kind == KIND_BAND ? "band." : "",
                tune_name(t[k].prec), t[k].kb, t[k].rb, t[k].value);
    fprintf(f, "\n}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), path) != 0) return fail(c, CPMI_ERR_ARG, "cannot write %s", path);
    return CPMI_OK;
}

int cpmi_tune_lookup(cpmi_ctx *c, int dtype, int precision, int64_t d, double pairs, int32_t *prec_out,
                     int32_t *tile_out)
{
    if (!c || !prec_out || !tile_out) return CPMI_ERR_ARG;
    const int p = resolve_prec(c, dtype, precision, d, pairs);
    if (p < 0) return p;
    *prec_out = p;
    *tile_out = pick_tile(c, p, d, pairs);
    return CPMI_OK;
}

int cpmi_tune_lookup_band(cpmi_ctx *c, int precision, int64_t d, double pairs, int32_t *band_out)
{
    if (!c || !band_out) return CPMI_ERR_ARG;
    if (precision != CPMI_PREC_F32 && precision != CPMI_PREC_BF16 && precision != CPMI_PREC_I8)
        return fail(c, CPMI_ERR_ARG, "precision must be F32, BF16 or I8");
    *band_out = pick_band(c, precision, d, pairs);
    return CPMI_OK;
}

// ---- debug entry points (declared in cpmi_debug.h) ------------------------

int64_t cpmi_dbg_tile_list(int64_t n, int64_t excl, int tile, uint64_t *out, int64_t cap)
{
    if (n < 0 || excl < 1 || (tile != 128 && tile != 256)) return CPMI_ERR_ARG;
    std::vector<HostProb> hp(1);
    hp[0].n = n;
    hp[0].excl = excl;
    std::vector<uint64_t> tl;
    int64_t nf = 0;
    build_tiles(hp, tile, tl, &nf);
    for (int64_t k = 0; k < (int64_t)tl.size() && k < cap; ++k) out[k] = tl[k];
    return (int64_t)tl.size();
}

int64_t cpmi_dbg_tile_list_two(int64_t na, int64_t nb, int64_t split, int tile, uint64_t *out, int64_t cap,
                               int64_t *nfull)
{
    if (na < 0 || nb < 0 || split < na || split % 256 || (tile != 128 && tile != 256)) return CPMI_ERR_ARG;
    std::vector<HostProb> hp(1);
    hp[0].n = split + nb;
    hp[0].split = split;
    hp[0].na = na;
    std::vector<uint64_t> tl;
    int64_t nf = 0;
    build_tiles(hp, tile, tl, &nf);
    for (int64_t k = 0; k < (int64_t)tl.size() && k < cap; ++k) out[k] = tl[k];
    if (nfull) *nfull = nf;
    return (int64_t)tl.size();
}

int cpmi_dbg_copy(void *dst, const void *src, int64_t bytes, void *stream)
{
    if (!dst || !src || bytes < 0 || bytes % 16) return CPMI_ERR_ARG;
    const char *a = (const char *)src, *b = (const char *)dst;
    if (a < b + bytes && b < a + bytes) return CPMI_ERR_ARG;
    launch_calib_copy(src, dst, bytes / 16, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) return CPMI_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return CPMI_ERR_HIP;
    return CPMI_OK;
}

int64_t cpmi_dbg_pruned_tiles(int64_t n, int tile, int q, const double *lo, const double *hi, double T, int64_t band,
                              uint64_t *out, int64_t cap, int64_t *nfull, int64_t *npruned)
{
    if (n < 2 || (tile != 128 && tile != 256) || q < 1 || q > 32 || !lo || !hi || cap < 0 || (cap > 0 && !out))
        return CPMI_ERR_ARG;
    const int64_t nT = (n + tile - 1) / tile;
    HostProb h;
    h.n = n;
    h.excl = 1;
    std::vector<double> vlo(lo, lo + nT * q), vhi(hi, hi + nT * q);
    std::vector<uint64_t> tl;
    int64_t nf = 0, np = 0;
    pruned_tiles(h, tile, q, vlo, vhi, T, band, tl, nf, np);
    for (int64_t k = 0; k < (int64_t)tl.size() && k < cap; ++k) out[k] = tl[(size_t)k];
    if (nfull) *nfull = nf;
    if (npruned) *npruned = np;
    return (int64_t)tl.size();
}

int64_t cpmi_dbg_pruned_tiles_gpu(cpmi_ctx *c, int64_t n, int tile, int q, const double *lo, const double *hi, double T,
                                  int64_t excl, int permuted, uint64_t *out, int64_t cap, int64_t *nfull,
                                  int64_t *npruned, void *stream)
{
    if (!c) return CPMI_ERR_ARG;
    if (n < 2 || n > ((int64_t)1 << 31) - 1 || (tile != 128 && tile != 256) || q < 1 || q > 32 || !lo || !hi ||
        cap < 0 || (cap > 0 && !out) || excl < 1 || excl > ((int64_t)1 << 30))
        return fail(c, CPMI_ERR_ARG, "bad arguments");
    hipSetDevice(c->device);
    const hipStream_t st = (hipStream_t)stream;
    const int64_t nT = (n + tile - 1) / tile;
    int rc;
    if ((rc = ensure(c, c->mlo, (size_t)nT * q * 8))) return rc;
    if ((rc = ensure(c, c->mhi, (size_t)nT * q * 8))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->mlo.p, lo, (size_t)nT * q * 8, hipMemcpyHostToDevice, st));
    HIPCHK(c, hipMemcpyAsync(c->mhi.p, hi, (size_t)nT * q * 8, hipMemcpyHostToDevice, st));
    HostProb h;
    h.n = n;
    h.excl = excl;
    h.motif = permuted != 0;
    static const int32_t any_perm = 0;
    h.perm = permuted ? &any_perm : nullptr;   // only its presence counts here
    if ((rc = queue_prune_list(c, h, tile, q, T, nullptr, 0.0, st))) return rc;
    HIPCHK(c, hipStreamSynchronize(st));
    const DevList dl = prune_list_of(c);
    const int64_t m = std::min(cap, dl.ntiles);
    if (m > 0) HIPCHK(c, hipMemcpy(out, dl.tiles, (size_t)m * 8, hipMemcpyDeviceToHost));
    if (nfull) *nfull = dl.nfull;
    if (npruned) *npruned = nT * (nT + 1) / 2 - (c->plist[2] + c->plist[3]);
    return dl.ntiles;
}

int cpmi_dbg_set_prune_order(cpmi_ctx *c, int order, double w)
{
    if (!c || order < 0 || order > 1 || !(w > 0.0) || !std::isfinite(w)) return CPMI_ERR_ARG;
    c->prune_order = order;
    c->prune_w = w;
    return CPMI_OK;
}

double cpmi_dbg_tile_lb(const double *loI, const double *hiI, const double *loJ, const double *hiJ, int q)
{
    if (!loI || !hiI || !loJ || !hiJ || q < 1) return -1.0;
    return tile_lower_bound(loI, hiI, loJ, hiJ, q);
}

int cpmi_dbg_tune(const char *cache_in, const char *cache_out, int ncu, int dtype, int precision, int64_t d,
                  double pairs, int32_t *prec_out, int32_t *tile_out)
{
    if (ncu < 1) return CPMI_ERR_ARG;
    cpmi_ctx c;  // host state only: no stream, event or buffer is created
    c.ncu = ncu;
    load_tune_cache(&c, cache_in);
    int rc = CPMI_OK;
    if (cache_out) rc = cpmi_save_tune_cache(&c, cache_out);
    if (rc == CPMI_OK) rc = cpmi_tune_lookup(&c, dtype, precision, d, pairs, prec_out, tile_out);
    return rc;
}

int64_t cpmi_dbg_xs_offset256(int64_t row, int64_t byte, int64_t rowbytes)
{
    if (row < 0 || byte < 0 || rowbytes <= 0 || rowbytes % (2 * l256::SLICE) || byte >= rowbytes) return -1;
    return l256::xs_offset(row, byte, rowbytes);
}

int cpmi_dbg_layout256(int wave, int q, int lane, int32_t *out4)
{
    if (wave < 0 || wave > 3 || q < 0 || q >= l256::NQ || lane < 0 || lane > 63 || !out4) return CPMI_ERR_ARG;
    out4[0] = l256::dma_row(wave, q, lane);
    out4[1] = l256::dma_col(wave, q, lane);
    out4[2] = l256::dma_lds(wave, q, lane);
    out4[3] = l256::frag_lds(out4[0], out4[1] >> 4);
    return CPMI_OK;
}

double cpmi_dbg_tile_bound(const float *bI, const float *bJ, int32_t kpad, int64_t d, int precision, int form)
{
    return tile_bound(make_float4(bI[0], bI[1], bI[2], bI[3]), make_float4(bJ[0], bJ[1], bJ[2], bJ[3]), kpad, d,
                      precision, form);
}

double cpmi_dbg_mfma_peak(int device, int precision, int iters, double *ms_out)
{
    if (precision < 1 || precision > 3 || iters < 1) return CPMI_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return CPMI_ERR_HIP;
    int ncu = 256;
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    const int prec = precision == CPMI_PREC_F32 ? P_F32 : (precision == CPMI_PREC_BF16 ? P_BF16 : P_I8);
    float *out = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc(&out, (size_t)ncu * 256 * sizeof(float)) != hipSuccess) return CPMI_ERR_HIP;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    launch_mfma_peak(prec, 2, ncu, out, nullptr);   // warm-up
    hipEventRecord(e0, nullptr);
    launch_mfma_peak(prec, iters, ncu, out, nullptr);
    hipEventRecord(e1, nullptr);
    const hipError_t e = hipEventSynchronize(e1);
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(out);
    if (e != hipSuccess || !(ms > 0.f)) return CPMI_ERR_HIP;
    if (ms_out) *ms_out = ms;
    // operations of one accumulation step: 32 x 32 outputs times K (8 = four FP32 instructions, 16, 32),
    // two per multiply-add
    const double per = prec == P_F32 ? 32.0 * 32 * 8 * 2 : (prec == P_BF16 ? 32.0 * 32 * 16 * 2 : 32.0 * 32 * 32 * 2);
    const double ops = (double)ncu * 4 * 16 * (double)iters * per;
    return ops / (ms * 1e-3) / 1e12;
}

int cpmi_dbg_mfma_probe(int precision, const void *A, const void *B, float *C, void *stream)
{
    if (precision < 1 || precision > 3 || !A || !B || !C) return CPMI_ERR_ARG;
    launch_mfma_probe(precision, A, B, C, (hipStream_t)stream);
    if (hipGetLastError() != hipSuccess) return CPMI_ERR_HIP;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return CPMI_ERR_HIP;
    return CPMI_OK;
}

int cpmi_dbg_screen_sample(cpmi_ctx *c, const void *src, int dtype, int64_t n, int64_t d, int64_t ld, int series,
                           int precision, int tile, const int64_t *tiles_ij, int64_t m, void *dump_out,
                           double *d2_out, double *bound_out, double *max_ratio_out, void *stream)
{
    if (!c) return CPMI_ERR_ARG;
    c->err.clear();
    if (!src || !tiles_ij || !dump_out || !d2_out || !bound_out || !max_ratio_out || m < 1)
        return fail(c, CPMI_ERR_ARG, "null argument or no tile");
    if (tile != 128 && tile != 256) return fail(c, CPMI_ERR_ARG, "tile must be 128 or 256");
    if (dtype != CPMI_F32 && dtype != CPMI_I8) return fail(c, CPMI_ERR_ARG, "unknown dtype");
    if (series && (dtype != CPMI_F32 || d < 2 || n < d || d > SERIES_MAX_ELL))
        return fail(c, CPMI_ERR_ARG, "series: float32, 2 <= ell <= len");
    if (!series && (d < 1 || ld < d || n < 1)) return fail(c, CPMI_ERR_ARG, "bad shape");
    if (dtype == CPMI_I8 && precision != CPMI_PREC_I8 && precision != CPMI_PREC_AUTO)
        return fail(c, CPMI_ERR_ARG, "int8 points take CPMI_PREC_I8");
    const int64_t rows = series ? n - d + 1 : n;
    const int prec = resolve_prec(c, dtype, precision, d, (double)pairs_of(rows, 1));
    if (prec < 0) return prec;
    const int64_t nT = (rows + tile - 1) / tile;
    std::vector<uint64_t> tl((size_t)m);
    for (int64_t t = 0; t < m; ++t) {
        const int64_t I = tiles_ij[2 * t], J = tiles_ij[2 * t + 1];
        if (I < 0 || J < 0 || I >= nT || J >= nT) return fail(c, CPMI_ERR_ARG, "tile (%lld, %lld) out of range", (long long)I, (long long)J);
        tl[(size_t)t] = tile_pack(0, (uint32_t)I, (uint32_t)J);
    }
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    std::vector<HostProb> hp(1);
    hp[0].n = rows;
    hp[0].d = d;
    hp[0].ld = series ? 1 : ld;
    hp[0].excl = series ? d : 1;
    hp[0].motif = series ? 1 : 0;
    hp[0].src = src;
    hp[0].src_i8 = dtype == CPMI_I8;
    hp[0].len = series ? n : 0;
    // per-tile bounds and the ratio word: a small buffer of its own (test only)
    DevBuf eb;
    HIPCHK(c, hipMalloc(&eb.p, (size_t)m * 8 + 256));
    DumpReq dr{dump_out, d2_out, (double *)eb.p, (unsigned int *)((char *)eb.p + (size_t)m * 8)};
    RunOut ro;
    rc = run_search(c, hp, prec, tile, false, false, st, false, ro, &tl, 0, false, {}, nullptr, &dr);
    unsigned int rbits = 0;
    if (rc == CPMI_OK) {
        hipError_t e = hipMemcpy(bound_out, eb.p, (size_t)m * 8, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(&rbits, dr.ratio, 4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(c, CPMI_ERR_HIP, "copy of the bounds failed: %s", hipGetErrorString(e));
    }
    hipFree(eb.p);
    if (rc) return rc;
    if ((rc = flags_error(c, ro.res[0].flags))) return rc;
    *max_ratio_out = (double)__builtin_bit_cast(float, rbits);
    return CPMI_OK;
}

int cpmi_dbg_znorm(cpmi_ctx *c, const float *series, int64_t len, int64_t ell, int precision, double *mu,
                   double *sigma, void *stream)
{
    if (!c || !series || !mu || !sigma || ell < 2 || len < ell) return CPMI_ERR_ARG;
    const int prec = resolve_prec(c, CPMI_F32, precision, ell, (double)pairs_of(len - ell + 1, ell));
    if (prec < 0) return prec;
    int rc;
    if ((rc = set_device(c))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t N = len - ell + 1;
    const int32_t kpad = kpad_for(prec, ell, 128);
    const int64_t npad = (N + 255) / 256 * 256;
    if ((rc = ensure(c, c->w.xs, (size_t)npad * kpad * elem_bytes(prec)))) return rc;
    if ((rc = ensure(c, c->w.shat, (size_t)npad * 4))) return rc;
    if ((rc = ensure(c, c->w.bmax, (size_t)(npad / 128) * 16))) return rc;
    if ((rc = ensure(c, c->w.res, sizeof(ResDev)))) return rc;
    if ((rc = ensure(c, c->w.jobs, sizeof(SeriesJob)))) return rc;
    SeriesJob j;
    memset(&j, 0, sizeof j);
    j.T = series;
    j.len = len;
    j.ell = ell;
    j.npad = npad;
    j.blk_base = 0;
    j.xs = c->w.xs.p;
    j.shat = c->w.shat.p;
    j.bmax = (float4 *)c->w.bmax.p;
    j.mu = mu;
    j.sigma = sigma;
    j.flags = &((ResDev *)c->w.res.p)->flags;
    j.kpad = kpad;
    HIPCHK(c, hipMemcpyAsync(c->w.jobs.p, &j, sizeof j, hipMemcpyHostToDevice, st));
    launch_reset_res((ResDev *)c->w.res.p, 1, st);
    launch_fill_u32((uint32_t *)c->w.bmax.p, 0u, (npad / 128) * 4, st);
    launch_prep_series((const SeriesJob *)c->w.jobs.p, 1, npad / SERIES_WPB, prec, 128, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    return CPMI_OK;
}

}  // extern "C"
