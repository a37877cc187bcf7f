// From screen to exact answer.
//
// 1. reduce_U / select: U[p] = min over tiles of (tile minimum + bound) is a
//    proven upper bound of the least canonical d^2; a tile can hold the
//    minimum only if (tile minimum - bound) <= U[p], so only those tiles are
//    screened a second time (this mirrors the paper's two-phase structure,
//    Section 3.6: cheap elimination first, exact evaluation of the survivors).
// 2. verify: every emitted candidate gets its canonical d^2 (ascending-k fma on
//    double differences; for windows the canonical z-normalised values are
//    rebuilt from T, mu and sigma; exact int64 for int8) -- the "compute
//    d(p_i, p_j)" step of MPR and MPR-FRNNS.
// 3. closest pair: least d^2, ties to the lexicographically smallest (i, j);
//    radius: keep d^2 <= R^2 (MPR-FRNNS step 5), sort by (i, j).
//
// Compiled with -ffp-contract=off so the FP64 sequence matches the canonical
// definition operation for operation.
#include <rocprim/device/device_radix_sort.hpp>

#include "bound.h"
#include "cpmi_internal.h"

namespace cpmi {

__device__ __forceinline__ double tile_min_value(uint32_t bits, int prec)
{
    return prec == P_I8 ? (double)(int)bits : (double)__uint_as_float(bits);
}

// Minimum screen value of list entry t: the least of its four waves' minima.
__device__ __forceinline__ double tile_min_of(const uint32_t *tile_min, int64_t t, int prec)
{
    const uint4 w = *(const uint4 *)(tile_min + 4 * t);
    return fmin(fmin(tile_min_value(w.x, prec), tile_min_value(w.y, prec)),
                fmin(tile_min_value(w.z, prec), tile_min_value(w.w, prec)));
}

__device__ __forceinline__ double tile_bound_of(const Prob &P, int64_t I, int64_t J, int prec)
{
    if (prec == P_I8) return 0.0;
    return tile_bound(P.bmax[I], P.bmax[J], P.kpad, P.d, prec, P.form);
}

// Each wave takes 64 consecutive list entries per step; when they all belong
// to one problem (always for a single problem, and inside each problem's run
// of a batched list) the wave reduces in registers and one lane keeps a
// running minimum. At the end the work-group's waves merge their minima per
// problem in LDS, so the global atomic is hit about once per work-group and
// problem. Work-groups of 1024 threads, a few steps per wave: enough waves to
// cover the list in a few steps without many atomics on one address.
constexpr int RU_THREADS = 1024;
__global__ __launch_bounds__(RU_THREADS) void reduce_U_kernel(const Prob *probs, const uint64_t *tiles,
                                                              int64_t ntiles, const uint32_t *tile_min, int prec,
                                                              unsigned long long *Ubits)
{
    __shared__ uint32_t wp[RU_THREADS / 64];
    __shared__ unsigned long long wv[RU_THREADS / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    uint32_t cur_p = 0xffffffffu;
    unsigned long long cur = ~0ull;  // running min of this wave (lane 0)
    for (int64_t base = wid * 64; base < ntiles; base += nw * 64) {
        const int64_t t = base + lane;
        uint32_t p = 0xffffffffu;
        unsigned long long ub_bits = ~0ull;
        if (t < ntiles) {
            const uint64_t e = tiles[t];
            if (e != TILE_NONE) {
                p = tile_prob(e);
                const double m = tile_min_of(tile_min, t, prec);
                if (m == m && !isinf(m)) {
                    const Prob &P = probs[p];
                    const double E = tile_bound_of(P, tile_I(e), tile_J(e), prec);
                    double ub = m + E;
                    ub += add_margin(m, E);
                    if (!(ub > 0.0)) ub = 0.0;
                    ub_bits = (unsigned long long)__double_as_longlong(ub);
                }
            }
        }
        // one problem in the whole wave (entries without one do not count)?
        uint32_t p0 = p;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) p0 = min(p0, (uint32_t)__shfl_xor((int)p0, o, 64));
        const bool uniform = __all(p == p0 || p == 0xffffffffu);
        if (uniform) {
            unsigned long long m = ub_bits;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const unsigned long long other = __shfl_xor(m, o, 64);
                m = other < m ? other : m;
            }
            if (lane == 0 && p0 != 0xffffffffu) {
                if (p0 != cur_p) {
                    if (cur_p != 0xffffffffu && cur != ~0ull) atomicMin(&Ubits[cur_p], cur);
                    cur_p = p0;
                    cur = m;
                } else if (m < cur) {
                    cur = m;
                }
            }
        } else if (p != 0xffffffffu && ub_bits != ~0ull) {
            atomicMin(&Ubits[p], ub_bits);
        }
    }
    if (lane == 0) {
        wp[wave] = cur != ~0ull ? cur_p : 0xffffffffu;
        wv[wave] = cur;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // the waves' last problems, merged where neighbours share one
        uint32_t p = 0xffffffffu;
        unsigned long long v = ~0ull;
        for (int w = 0; w < RU_THREADS / 64; ++w) {
            if (wp[w] == 0xffffffffu) continue;
            if (wp[w] != p) {
                if (p != 0xffffffffu) atomicMin(&Ubits[p], v);
                p = wp[w];
                v = wv[w];
            } else if (wv[w] < v) {
                v = wv[w];
            }
        }
        if (p != 0xffffffffu) atomicMin(&Ubits[p], v);
    }
}

// The selected tiles twice: appended to sel (any order), and in place of the
// list in dense (list order, TILE_NONE elsewhere), which keeps the list's
// locality when many tiles are selected.
__global__ void select_kernel(const Prob *probs, const uint64_t *tiles, int64_t ntiles, const uint32_t *tile_min,
                              int prec, const unsigned long long *Ubits, uint64_t *sel, u64c *sel_count,
                              uint64_t *dense)
{
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < ntiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t e = tiles[t];
        dense[t] = TILE_NONE;
        if (e == TILE_NONE) continue;
        const uint32_t p = tile_prob(e);
        const Prob &P = probs[p];
        const double m = tile_min_of(tile_min, t, prec);
        if (!(m == m) || isinf(m)) continue;
        const double E = tile_bound_of(P, tile_I(e), tile_J(e), prec);
        double lb = m - E;
        lb -= add_margin(m, E);
        bool want = false;
        if (Ubits) want = lb <= __longlong_as_double((long long)Ubits[p]);
        if (P.r2 >= 0.0) want = want || lb <= P.r2;
        if (want) {
            const u64c k = atomicAdd(sel_count, 1ull);
            sel[k] = e;
            dense[t] = e;
        }
    }
}

static unsigned grid_of(int64_t n)
{
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (unsigned)g;
}

void launch_reduce_U(const Prob *probs, const uint64_t *tiles, int64_t ntiles, const uint32_t *tile_min, int prec,
                     unsigned long long *Ubits, hipStream_t st)
{
    int64_t g = (ntiles + RU_THREADS * 2 - 1) / (RU_THREADS * 2);   // about 2 steps per wave
    g = g < 1 ? 1 : (g > 1024 ? 1024 : g);
    hipLaunchKernelGGL(reduce_U_kernel, dim3((unsigned)g), dim3(RU_THREADS), 0, st, probs, tiles, ntiles, tile_min,
                       prec, Ubits);
}

void launch_select(const Prob *probs, const uint64_t *tiles, int64_t ntiles, const uint32_t *tile_min, int prec,
                   const unsigned long long *Ubits, uint64_t *sel, u64c *sel_count, uint64_t *dense, hipStream_t st)
{
    hipLaunchKernelGGL(select_kernel, dim3(grid_of(ntiles)), dim3(256), 0, st, probs, tiles, ntiles, tile_min, prec,
                       Ubits, sel, sel_count, dense);
}

// ---------------------------------------------------------------------------
// canonical squared distance, one wave per pair: the lanes form 64
// consecutive terms at a time (loads and normalisations in parallel), and
// every lane then adds them in order, broadcast lane by lane, so the sum is
// the sequential FP64 sum over k = 0 .. d-1. The next 64 terms are formed
// before the current ones are added.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lane_value(double v, int u)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, u);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), u);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ double canonical_d2(const Prob &P, int64_t i, int64_t j, int lane)
{
    const int64_t d = P.d;
    if (P.src_i8) {
        // exact integer sum: any order
        const signed char *x = (const signed char *)P.src + i * P.ld;
        const signed char *y = (const signed char *)P.src + j * P.ld;
        long long acc = 0;
        for (int64_t k = lane; k < d; k += 64) {
            const long long t = (long long)x[k] - (long long)y[k];
            acc += t * t;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        return (double)acc;
    }
    const float *T = (const float *)P.src;
    const float *x = T + i * P.ld, *y = T + j * P.ld;
    double mi = 0.0, si = 1.0, mj = 0.0, sj = 1.0;
    if (P.motif) {
        mi = P.mu[i], si = P.sigma[i], mj = P.mu[j], sj = P.sigma[j];
        x = T + i;
        y = T + j;
    }
    auto term = [&](int64_t k) -> double {
        if (k >= d) return 0.0;
        if (P.motif) return ((double)x[k] - mi) / si - ((double)y[k] - mj) / sj;
        return (double)x[k] - (double)y[k];
    };
    double acc = 0.0;
    double t = term(lane);
    for (int64_t c0 = 0; c0 < d; c0 += 64) {
        const double tn = term(c0 + 64 + lane);
        if (c0 + 64 <= d) {
#pragma unroll
            for (int u = 0; u < 64; ++u) {
                const double tu = lane_value(t, u);
                acc = fma(tu, tu, acc);
            }
        } else {
            for (int u = 0; u < (int)(d - c0); ++u) {
                const double tu = lane_value(t, u);
                acc = fma(tu, tu, acc);
            }
        }
        t = tn;
    }
    return acc;
}

// Source rows (a < b) of a candidate, whose screen rows may be permuted.
__device__ __forceinline__ void cand_rows(const Prob &P, const Cand &cd, int64_t &a, int64_t &b)
{
    const int64_t x = src_row(P, cd.i), y = src_row(P, cd.j);
    a = x < y ? x : y;
    b = x < y ? y : x;
}

// Screening-error maxima of the candidates a wave verified, merged into the
// problem's result with one set of atomics per run of one problem (lane 0).
struct ErrAcc {
    uint32_t p = 0xffffffffu;
    float err = 0.f, ratio = 0.f, bound = 0.f;
    __device__ void flush(ResDev *res)
    {
        if (p == 0xffffffffu) return;
        atomicMax(&res[p].err_bits, __float_as_uint(err));
        if (bound > 0.f) {
            atomicMax(&res[p].ratio_bits, __float_as_uint(ratio));
            atomicMax(&res[p].bound_bits, __float_as_uint(bound));
        }
    }
    __device__ void add(ResDev *res, uint32_t q, double dt, double d2, double E)
    {
        if (q != p) {
            flush(res);
            p = q;
            err = ratio = bound = 0.f;
        }
        const double e = fabs(dt - d2);
        err = fmaxf(err, f32_up(e));
        if (E > 0.0) {
            ratio = fmaxf(ratio, f32_up(e / E));
            bound = fmaxf(bound, f32_up(E));
        }
    }
};

// One wave per candidate (4 per work-group); each wave keeps the least d2
// and the error maxima of the run of candidates of one problem it verified
// and merges them with one set of atomics per run.
__global__ __launch_bounds__(256) void verify_cpp_kernel(const Prob *probs, const Cand *cand, const u64c *cnt,
                                                         uint64_t cap, int prec, int tile, double *cand_d2,
                                                         ResDev *res)
{
    const int64_t m = min((int64_t)*cnt, (int64_t)cap);
    const int lane = threadIdx.x & 63;
    ErrAcc ea;
    uint32_t bp = 0xffffffffu;
    unsigned long long bbits = ~0ull;
    for (int64_t c = blockIdx.x * 4 + (threadIdx.x >> 6); c < m; c += (int64_t)gridDim.x * 4) {
        const Cand cd = cand[c];
        const Prob &P = probs[cd.p];
        int64_t a, b;
        cand_rows(P, cd, a, b);
        const double d2 = canonical_d2(P, a, b, lane);
        if (lane == 0) {
            cand_d2[c] = d2;
            if (cd.p != bp) {
                if (bp != 0xffffffffu) atomicMin(&res[bp].best_d2, bbits);
                bp = cd.p;
                bbits = ~0ull;
            }
            const unsigned long long bits = (unsigned long long)__double_as_longlong(d2);
            bbits = bits < bbits ? bits : bbits;   // d2 >= 0: the bits order as the values
            ea.add(res, cd.p, (double)cd.dt, d2, tile_bound_of(P, cd.i / tile, cd.j / tile, prec));
        }
    }
    if (lane == 0) {
        if (bp != 0xffffffffu) atomicMin(&res[bp].best_d2, bbits);
        ea.flush(res);
    }
}

__global__ void pick_cpp_kernel(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap,
                                const double *cand_d2, ResDev *res)
{
    const int64_t m = min((int64_t)*cnt, (int64_t)cap);
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < m; c += (int64_t)gridDim.x * blockDim.x) {
        const Cand cd = cand[c];
        if ((unsigned long long)__double_as_longlong(cand_d2[c]) == res[cd.p].best_d2) {
            int64_t a, b;
            cand_rows(probs[cd.p], cd, a, b);
            atomicMin(&res[cd.p].best_ij, ((unsigned long long)(unsigned)a << 32) | (unsigned)b);
        }
    }
}

// The canonical d2 of rows i and j computed by one lane alone: the same
// terms in the same ascending order as canonical_d2, with no broadcasts
// (each lane of a wave runs its own candidate).
__device__ double canonical_d2_lane(const Prob &P, int64_t i, int64_t j)
{
    const int64_t d = P.d;
    if (P.src_i8) {
        const signed char *x = (const signed char *)P.src + i * P.ld;
        const signed char *y = (const signed char *)P.src + j * P.ld;
        long long acc = 0;
        for (int64_t k = 0; k < d; ++k) {
            const long long t = (long long)x[k] - (long long)y[k];
            acc += t * t;
        }
        return (double)acc;
    }
    const float *T = (const float *)P.src;
    double acc = 0.0;
    if (P.motif) {
        const float *x = T + i, *y = T + j;
        const double mi = P.mu[i], si = P.sigma[i], mj = P.mu[j], sj = P.sigma[j];
        for (int64_t k = 0; k < d; ++k) {
            const double t = ((double)x[k] - mi) / si - ((double)y[k] - mj) / sj;
            acc = fma(t, t, acc);
        }
        return acc;
    }
    const float *x = T + i * P.ld, *y = T + j * P.ld;
    int64_t k = 0;
    if ((((uintptr_t)x | (uintptr_t)y) & 15) == 0) {
        // 16-byte loads, the terms still taken one at a time in order
        for (; k + 4 <= d; k += 4) {
            const float4 u = *(const float4 *)(x + k), w = *(const float4 *)(y + k);
            double t = (double)u.x - (double)w.x;
            acc = fma(t, t, acc);
            t = (double)u.y - (double)w.y;
            acc = fma(t, t, acc);
            t = (double)u.z - (double)w.z;
            acc = fma(t, t, acc);
            t = (double)u.w - (double)w.w;
            acc = fma(t, t, acc);
        }
    }
    for (; k < d; ++k) {
        const double t = (double)x[k] - (double)y[k];
        acc = fma(t, t, acc);
    }
    return acc;
}

// One lane per candidate: at volume (millions of candidates) 64 chains in
// flight per wave hide the FP64 latency that one chain per wave exposes. The
// pairs within the radius get their output slots with one atomic add per
// wave step, and the error maxima are merged with one set of atomics per
// wave (all lanes of one problem) or per lane.
__global__ __launch_bounds__(256) void verify_frnn_kernel(const Prob *probs, const Cand *cand, const u64c *cnt,
                                                          uint64_t cap, int prec, int tile, uint64_t *keys,
                                                          double *vals, u64c *out_cnt, uint64_t out_cap,
                                                          ResDev *res)
{
    const int64_t m = min((int64_t)*cnt, (int64_t)cap);
    const int lane = threadIdx.x & 63;
    const int64_t wid = blockIdx.x * 4 + (threadIdx.x >> 6), nw = (int64_t)gridDim.x * 4;
    ErrAcc ea;
    for (int64_t base = wid * 64; base < m; base += nw * 64) {
        const int64_t c = base + lane;
        uint64_t key = 0;
        double d2 = 0.0;
        uint32_t in = 0;
        if (c < m) {
            const Cand cd = cand[c];
            // not an unused slot of a screen wave's slab, nor a pair that the
            // bound of its own two rows (tighter than the tile's, which
            // emitted it) puts outside the radius: |D~ - d2| <= E_ij, so
            // d2 <= R2 needs D~ - E_ij <= R2 (with the selection's margin)
            bool live = cd.p != 0xffffffffu;
            if (live && probs[cd.p].rowstat) {
                const Prob &P = probs[cd.p];
                const double E = tile_bound(P.rowstat[cd.i], P.rowstat[cd.j], P.kpad, P.d, prec, P.form);
                const double dt = (double)cd.dt;
                double lb = dt - E;
                lb -= add_margin(dt, E);
                live = lb <= P.r2;
            }
            if (live) {
                const Prob &P = probs[cd.p];
                int64_t a, b;
                cand_rows(P, cd, a, b);
                d2 = canonical_d2_lane(P, a, b);
                // the bound is indexed by screen-row blocks
                ea.add(res, cd.p, (double)cd.dt, d2, tile_bound_of(P, cd.i / tile, cd.j / tile, prec));
                key = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
                in = d2 <= P.r2;
            }
        }
        const uint64_t k = wave_reserve(out_cnt, in);
        if (in && k < out_cap) {
            keys[k] = key;
            vals[k] = d2;
        }
    }
    // one problem in every lane (or none): the wave's maxima, one lane merges them
    const uint32_t p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)ea.p);
    if (__all(ea.p == p0 || ea.p == 0xffffffffu)) {
        float e = ea.err, r = ea.ratio, bd = ea.bound;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            e = fmaxf(e, __shfl_xor(e, o, 64));
            r = fmaxf(r, __shfl_xor(r, o, 64));
            bd = fmaxf(bd, __shfl_xor(bd, o, 64));
        }
        if (lane == 0 && p0 != 0xffffffffu) {
            ea.p = p0;
            ea.err = e;
            ea.ratio = r;
            ea.bound = bd;
            ea.flush(res);
        }
    } else {
        ea.flush(res);
    }
}

// Windows of a series, few candidates (motifs, pruned searches): each term
// of the canonical sum needs two FP64 divisions, and the sum is one chain of
// d dependent additions. A lane per candidate leaves most of the chip idle
// when there are only thousands of candidates; a wave per candidate spends
// most of its instructions carrying the chain from lane to lane. Here a
// work-group takes 16 candidates at a time: for each chunk of 64 terms, the
// 16 threads of a candidate form 4 terms each into LDS, then one lane per
// candidate adds the chunk in ascending k (terms past d are exact zeros,
// which leave the sum as it is). The result is the canonical sum, bit for
// bit. FRNN (cand_d2 null): pairs within R2 are written as keys and values,
// candidates that the bound of their own two rows puts outside R2 are
// dropped first. Closest pair (keys null): d2 per candidate and the least
// one per problem, as verify_cpp_kernel.
constexpr int VW_C = 16;  // candidates per work-group and round
constexpr int VW_K = 64;  // terms per chunk

template <bool FRNN>
__global__ __launch_bounds__(256) void verify_windows_kernel(const Prob *probs, const Cand *cand, const u64c *cnt,
                                                             uint64_t cap, int prec, int tile, double *cand_d2,
                                                             uint64_t *keys, double *vals, u64c *out_cnt,
                                                             uint64_t out_cap, ResDev *res)
{
    __shared__ double sh_t[VW_C][VW_K + 1];
    __shared__ int32_t sh_live[VW_C];
    __shared__ int64_t sh_d[VW_C];
    const int64_t m = min((int64_t)*cnt, (int64_t)cap);
    const int tid = threadIdx.x, slot = tid >> 4, sub = tid & 15;
    ErrAcc ea;                       // chain lanes (tid < VW_C)
    uint32_t bp = 0xffffffffu;       // closest pair: the chain lane's run of one problem
    unsigned long long bbits = ~0ull;
    const int64_t ngroups = (m + VW_C - 1) / VW_C;
    for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
        // this thread's candidate (slot), its rows and window statistics
        const int64_t c = g * VW_C + slot;
        bool live = c < m;
        Cand cd{};
        if (live) {
            cd = cand[c];
            live = cd.p != 0xffffffffu;   // not an unused slot of a screen wave's slab
        }
        if (FRNN && live && probs[cd.p].rowstat) {
            const Prob &P = probs[cd.p];
            const double E = tile_bound(P.rowstat[cd.i], P.rowstat[cd.j], P.kpad, P.d, prec, P.form);
            const double dt = (double)cd.dt;
            double lb = dt - E;
            lb -= add_margin(dt, E);
            live = lb <= P.r2;
        }
        const float *x = nullptr, *y = nullptr;
        double mi = 0.0, si = 1.0, mj = 0.0, sj = 1.0;
        int64_t d = 0;
        bool motif = false;
        if (live) {
            const Prob &P = probs[cd.p];
            int64_t a, b;
            cand_rows(P, cd, a, b);
            const float *T = (const float *)P.src;
            d = P.d;
            motif = P.motif != 0;
            if (motif) {
                x = T + a;
                y = T + b;
                mi = P.mu[a], si = P.sigma[a], mj = P.mu[b], sj = P.sigma[b];
            } else {
                x = T + a * P.ld;
                y = T + b * P.ld;
            }
        }
        if (sub == 0) {
            sh_live[slot] = live;
            sh_d[slot] = d;
        }
        __syncthreads();
        int64_t dmax = 0;
#pragma unroll
        for (int q = 0; q < VW_C; ++q) dmax = max(dmax, sh_d[q]);
        double acc = 0.0;   // chain lane tid: candidate g * VW_C + tid
        for (int64_t c0 = 0; c0 < dmax; c0 += VW_K) {
#pragma unroll
            for (int v = 0; v < VW_K / 16; ++v) {
                const int64_t k = c0 + sub + 16 * v;
                double t = 0.0;
                if (k < d)
                    t = motif ? ((double)x[k] - mi) / si - ((double)y[k] - mj) / sj : (double)x[k] - (double)y[k];
                sh_t[slot][sub + 16 * v] = t;
            }
            __syncthreads();
            if (tid < VW_C) {
#pragma unroll 16
                for (int u = 0; u < VW_K; ++u) {
                    const double tu = sh_t[tid][u];
                    acc = fma(tu, tu, acc);
                }
            }
            __syncthreads();
        }
        if (tid < 64) {
            // wave 0; its lanes below VW_C hold the sums of the group
            const int64_t cc = g * VW_C + tid;
            const bool mine = tid < VW_C && sh_live[tid];
            Cand ce{};
            if (mine) ce = cand[cc];
            const Prob *P = mine ? &probs[ce.p] : nullptr;
            int64_t a = 0, b = 0;
            if (mine) {
                cand_rows(*P, ce, a, b);
                ea.add(res, ce.p, (double)ce.dt, acc, tile_bound_of(*P, ce.i / tile, ce.j / tile, prec));
            }
            if constexpr (FRNN) {
                const bool in = mine && acc <= P->r2;
                const uint64_t k = wave_reserve(out_cnt, in);
                if (in && k < out_cap) {
                    keys[k] = ((uint64_t)(uint32_t)a << 32) | (uint32_t)b;
                    vals[k] = acc;
                }
            } else if (tid < VW_C && cc < m) {
                cand_d2[cc] = acc;
                if (mine) {
                    if (ce.p != bp) {
                        if (bp != 0xffffffffu) atomicMin(&res[bp].best_d2, bbits);
                        bp = ce.p;
                        bbits = ~0ull;
                    }
                    const unsigned long long bits = (unsigned long long)__double_as_longlong(acc);
                    bbits = bits < bbits ? bits : bbits;   // d2 >= 0: the bits order as the values
                }
            }
        }
        __syncthreads();   // sh_live, sh_d of the next group
    }
    if (tid < 64) {
        // one problem in every chain lane (or none): merged in the wave first
        const uint32_t p0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)ea.p);
        if (__all(ea.p == p0 || ea.p == 0xffffffffu)) {
            float e = ea.err, r = ea.ratio, bd = ea.bound;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                e = fmaxf(e, __shfl_xor(e, o, 64));
                r = fmaxf(r, __shfl_xor(r, o, 64));
                bd = fmaxf(bd, __shfl_xor(bd, o, 64));
            }
            if (tid == 0 && p0 != 0xffffffffu) {
                ea.p = p0;
                ea.err = e;
                ea.ratio = r;
                ea.bound = bd;
                ea.flush(res);
            }
        } else {
            ea.flush(res);
        }
        if constexpr (!FRNN) {
            const uint32_t q0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)bp);
            if (__all(bp == q0 || bp == 0xffffffffu)) {
                unsigned long long v = bbits;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    const unsigned long long w = __shfl_xor(v, o, 64);
                    v = w < v ? w : v;
                }
                if (tid == 0 && q0 != 0xffffffffu && v != ~0ull) atomicMin(&res[q0].best_d2, v);
            } else if (bp != 0xffffffffu) {
                atomicMin(&res[bp].best_d2, bbits);
            }
        }
    }
}

// One wave per dumped element (grid-stride over m tiles x tile^2 elements).
__global__ __launch_bounds__(256) void sample_check_kernel(const Prob *probs, const uint64_t *tiles, int64_t m,
                                                           int tile, const void *dump, int prec, double *d2_out,
                                                           double *E_out, unsigned int *ratio_bits)
{
    const int lane = threadIdx.x & 63;
    const int64_t per = (int64_t)tile * tile;
    for (int64_t e = blockIdx.x * 4 + (threadIdx.x >> 6); e < m * per; e += (int64_t)gridDim.x * 4) {
        const int64_t t = e / per, il = (e % per) / tile, jl = e % tile;
        const uint64_t ent = tiles[t];
        const Prob &P = probs[tile_prob(ent)];
        const int64_t gi = (int64_t)tile_I(ent) * tile + il, gj = (int64_t)tile_J(ent) * tile + jl;
        const double E = tile_bound_of(P, tile_I(ent), tile_J(ent), prec);
        if (lane == 0 && e % per == 0) E_out[t] = E;
        if (gi >= P.n || gj >= P.n) continue;
        const double d2 = canonical_d2(P, src_row(P, gi), src_row(P, gj), lane);
        if (lane == 0) {
            d2_out[e] = d2;
            const double dt = prec == P_I8 ? (double)((const int *)dump)[e] : (double)((const float *)dump)[e];
            const double err = fabs(dt - d2);
            const float ratio = prec == P_I8 ? (err == 0.0 ? 0.0f : INFINITY) : f32_up(err / E);
            atomicMax(ratio_bits, __float_as_uint(ratio));
        }
    }
}

void launch_sample_check(const Prob *probs, const uint64_t *tiles, int64_t m, int tile, const void *dump, int prec,
                         double *d2_out, double *E_out, unsigned int *ratio_bits, hipStream_t st)
{
    hipLaunchKernelGGL(sample_check_kernel, dim3(2048), dim3(256), 0, st, probs, tiles, m, tile, dump, prec, d2_out,
                       E_out, ratio_bits);
}

static unsigned verify_grid() { return 2048; }   // work-groups of 4 waves, a candidate per wave

void launch_verify_cpp(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, int prec, int tile,
                       double *cand_d2, ResDev *res, hipStream_t st)
{
    hipLaunchKernelGGL(verify_cpp_kernel, dim3(verify_grid()), dim3(256), 0, st, probs, cand, cnt, cap, prec, tile,
                       cand_d2, res);
}

void launch_pick_cpp(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, const double *cand_d2,
                     ResDev *res, hipStream_t st)
{
    hipLaunchKernelGGL(pick_cpp_kernel, dim3(256), dim3(256), 0, st, probs, cand, cnt, cap, cand_d2, res);
}

void launch_verify_windows(bool frnn, const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, int prec,
                           int tile, double *cand_d2, uint64_t *keys, double *vals, u64c *out_cnt, uint64_t out_cap,
                           ResDev *res, hipStream_t st)
{
    if (frnn)
        hipLaunchKernelGGL(verify_windows_kernel<true>, dim3(verify_grid()), dim3(256), 0, st, probs, cand, cnt, cap,
                           prec, tile, nullptr, keys, vals, out_cnt, out_cap, res);
    else
        hipLaunchKernelGGL(verify_windows_kernel<false>, dim3(verify_grid()), dim3(256), 0, st, probs, cand, cnt, cap,
                           prec, tile, cand_d2, nullptr, nullptr, nullptr, 0, res);
}

void launch_verify_frnn(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, int prec, int tile,
                        uint64_t *keys, double *vals, u64c *out_cnt, uint64_t out_cap, ResDev *res,
                        hipStream_t st)
{
    hipLaunchKernelGGL(verify_frnn_kernel, dim3(verify_grid()), dim3(256), 0, st, probs, cand, cnt, cap, prec, tile,
                       keys, vals, out_cnt, out_cap, res);
}

// ---------------------------------------------------------------------------
// bitonic sort of (key, value) pairs; mpad is a power of two. Stages with a
// partner distance below LOCAL run inside one work-group's LDS.
// ---------------------------------------------------------------------------
constexpr int LOCAL = 2048;  // elements per LDS block (1024 threads x 2)

__global__ void pad_sentinel_kernel(uint64_t *keys, double *vals, int64_t m, int64_t mpad)
{
    for (int64_t i = m + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mpad;
         i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = ~0ull;
        vals[i] = 0.0;
    }
}

__global__ void bitonic_global_kernel(uint64_t *keys, double *vals, int64_t mpad, int64_t k, int64_t j)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mpad; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t l = i ^ j;
        if (l > i) {
            const bool up = (i & k) == 0;
            const uint64_t a = keys[i], b = keys[l];
            if ((a > b) == up) {
                keys[i] = b;
                keys[l] = a;
                const double t = vals[i];
                vals[i] = vals[l];
                vals[l] = t;
            }
        }
    }
}

// Runs, for a fixed k, all stages j = jstart, jstart/2, ..., 1 on one LDS block.
__global__ __launch_bounds__(1024) void bitonic_local_kernel(uint64_t *keys, double *vals, int64_t k, int64_t jstart)
{
    __shared__ uint64_t sk[LOCAL];
    __shared__ double sv[LOCAL];
    const int64_t base = (int64_t)blockIdx.x * LOCAL;
    for (int q = threadIdx.x; q < LOCAL; q += 1024) {
        sk[q] = keys[base + q];
        sv[q] = vals[base + q];
    }
    __syncthreads();
    for (int64_t j = jstart; j > 0; j >>= 1) {
        for (int q = threadIdx.x; q < LOCAL; q += 1024) {
            const int l = q ^ (int)j;
            if (l > q) {
                const bool up = ((base + q) & k) == 0;
                const uint64_t a = sk[q], b = sk[l];
                if ((a > b) == up) {
                    sk[q] = b;
                    sk[l] = a;
                    const double t = sv[q];
                    sv[q] = sv[l];
                    sv[l] = t;
                }
            }
        }
        __syncthreads();
    }
    for (int q = threadIdx.x; q < LOCAL; q += 1024) {
        keys[base + q] = sk[q];
        vals[base + q] = sv[q];
    }
}

// The whole network in one work-group's LDS, for mpad <= LOCAL (one launch
// instead of one per stage).
__global__ __launch_bounds__(1024) void bitonic_small_kernel(uint64_t *keys, double *vals, int mpad)
{
    __shared__ uint64_t sk[LOCAL];
    __shared__ double sv[LOCAL];
    for (int q = threadIdx.x; q < mpad; q += 1024) {
        sk[q] = keys[q];
        sv[q] = vals[q];
    }
    __syncthreads();
    for (int k = 2; k <= mpad; k <<= 1)
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int q = threadIdx.x; q < mpad; q += 1024) {
                const int l = q ^ j;
                if (l > q) {
                    const bool up = (q & k) == 0;
                    const uint64_t a = sk[q], b = sk[l];
                    if ((a > b) == up) {
                        sk[q] = b;
                        sk[l] = a;
                        const double t = sv[q];
                        sv[q] = sv[l];
                        sv[l] = t;
                    }
                }
            }
            __syncthreads();
        }
    for (int q = threadIdx.x; q < mpad; q += 1024) {
        keys[q] = sk[q];
        vals[q] = sv[q];
    }
}

void launch_sort_pairs(uint64_t *keys, double *vals, int64_t m, int64_t mpad, hipStream_t st)
{
    if (m <= 1) return;
    if (mpad > m) hipLaunchKernelGGL(pad_sentinel_kernel, dim3(grid_of(mpad - m)), dim3(256), 0, st, keys, vals, m, mpad);
    if (mpad <= LOCAL) {
        hipLaunchKernelGGL(bitonic_small_kernel, dim3(1), dim3(1024), 0, st, keys, vals, (int)mpad);
        return;
    }
    for (int64_t k = 2; k <= mpad; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= LOCAL; j >>= 1)
            hipLaunchKernelGGL(bitonic_global_kernel, dim3(grid_of(mpad)), dim3(256), 0, st, keys, vals, mpad, k, j);
        if (mpad >= LOCAL) {
            hipLaunchKernelGGL(bitonic_local_kernel, dim3((unsigned)(mpad / LOCAL)), dim3(1024), 0, st, keys, vals, k, j);
        } else {
            for (; j > 0; j >>= 1)
                hipLaunchKernelGGL(bitonic_global_kernel, dim3(grid_of(mpad)), dim3(256), 0, st, keys, vals, mpad, k, j);
        }
    }
}

// Long lists: one rocPRIM radix sort of the (i << 32 | j) keys with the d2
// values, out of place (temp == nullptr: only sets *temp_bytes).
hipError_t sort_pairs_radix(void *temp, size_t *temp_bytes, const uint64_t *keys_in, uint64_t *keys_out,
                            const double *vals_in, double *vals_out, int64_t m, hipStream_t st)
{
    return rocprim::radix_sort_pairs(temp, *temp_bytes, keys_in, keys_out, vals_in, vals_out, (unsigned int)m, 0, 64,
                                     st);
}

__global__ void emit_pairs_kernel(const uint64_t *keys, const double *vals, int64_t m, int64_t *pairs, double *d2)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t k = keys[i];
        pairs[2 * i] = (int64_t)(k >> 32);
        pairs[2 * i + 1] = (int64_t)(k & 0xffffffffu);
        if (d2) d2[i] = vals[i];
    }
}

void launch_emit_pairs(const uint64_t *keys, const double *vals, int64_t m, int64_t *pairs, double *d2,
                       hipStream_t st)
{
    if (m > 0) hipLaunchKernelGGL(emit_pairs_kernel, dim3(grid_of(m)), dim3(256), 0, st, keys, vals, m, pairs, d2);
}

}  // namespace cpmi
