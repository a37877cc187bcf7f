// Persistent 256x256 Gram screen for CDNA4 (gfx950).
//
// Same contract as the 128-tile screen in screen.hip (pass 1: tile minimum of
// the screen value D~ = s^_i + s^_j - 2 <x~_i, x~_j>; pass 2: emission of the
// pairs within the closest-pair or radius thresholds), organised for
// throughput on large problems:
//   * a persistent grid walks the tile list with stride gridDim.x, so a
//     work-group keeps the slots of one XCD chunk of the list;
//   * K slices (128 bytes per row) go straight from global memory into LDS
//     with global_load_lds_dwordx4 (no staging registers), double-buffered,
//     one barrier per slice, and the first slice of the next tile is fetched
//     while the current tile's epilogue runs;
//   * each 8-row, 1 KB LDS block stores row r's 16-byte chunk c at slot
//     c ^ (r & 7), so the fragment reads of 8 consecutive rows hit 8
//     different bank groups;
//   * 4 waves in a 2x2 grid, each owning 128x128 outputs as 4x4 32x32 MFMA
//     blocks (256 accumulators per lane);
//   * the epilogue takes, per accumulator row, the minimum over the four
//     column blocks of s^_j - 2 G (one fma and half a min3 per element), adds
//     s^_i once per row, and only when the wave's minimum is within a
//     threshold scans the elements again to emit pairs.
#include "bound.h"
#include "cpmi_internal.h"
#include "layout256.h"

namespace cpmi {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void g_void;

namespace {

constexpr int T256 = 256;         // tile edge
constexpr int WT256 = 128;        // wave tile edge
constexpr int MB256 = 4;          // 32x32 blocks per wave edge
constexpr int SL = 128;           // K slice, bytes per row
constexpr int OPB = T256 * SL;    // one operand slice in LDS (32 KB)

template <int PREC> struct A2 { using T = f32x16; using S = float; };
template <> struct A2<P_I8> { using T = i32x16; using S = int; };

template <int PREC>
__device__ __forceinline__ void mma2(typename A2<PREC>::T &c, const u32x4 &a, const u32x4 &b)
{
    if constexpr (PREC == P_F32) {
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
    } else if constexpr (PREC == P_BF16) {
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                     0, 0, 0);
    } else {
        c = __builtin_amdgcn_mfma_i32_32x32x32_i8(__builtin_bit_cast(i32x4, a), __builtin_bit_cast(i32x4, b), c, 0,
                                                   0, 0);
    }
}

template <typename S> __device__ __forceinline__ S smin(S a, S b);
template <> __device__ __forceinline__ float smin(float a, float b) { return fminf(a, b); }
template <> __device__ __forceinline__ int smin(int a, int b) { return min(a, b); }

template <typename S> __device__ __forceinline__ S wmin(S v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = smin(v, __shfl_xor(v, o, 64));
    return v;
}

// s^_j - 2 g  (float: one fma; int8: exact int32)
__device__ __forceinline__ float part(float g, float sj) { return fmaf(-2.0f, g, sj); }
__device__ __forceinline__ int part(int g, int sj) { return sj - 2 * g; }

}  // namespace

// The two LDS stages are distinct __shared__ objects and every slice step
// names its stage at compile time, so the compiler can see that the
// direct-to-LDS loads into one stage never alias the fragment reads of the
// other and does not make those reads wait for the loads in flight.
__shared__ __attribute__((aligned(1024))) unsigned char g_stage0[2 * OPB];
__shared__ __attribute__((aligned(1024))) unsigned char g_stage1[2 * OPB];

template <int STG> __device__ __forceinline__ unsigned char *stage_ptr()
{
    return STG == 0 ? g_stage0 : g_stage1;
}

// Per-tile addressing of the direct-to-LDS loads: a uniform base per operand
// plus one 32-bit per-lane offset, so the loads use the scalar-base form and
// keep no 64-bit per-lane addresses live.
struct TileAddr {
    const unsigned char *ga;  // operand A rows of the tile (slice 0)
    const unsigned char *gb;  // operand B rows of the tile (slice 0)
    uint32_t lane_off;        // (wave*64 + ld_row) * rowbytes + ld_col
    uint32_t step8;           // 8 * rowbytes
    int nst;                  // K slices
};

template <int ESZ>
__device__ __forceinline__ TileAddr tile_addr(const ScreenArgs &args, uint64_t ent, int wave, int ld_row, int ld_col)
{
    const Prob &P = args.probs[tile_prob(ent)];
    const uint32_t rowbytes = (uint32_t)P.kpad * ESZ;
    const unsigned char *xs = (const unsigned char *)P.xs;
    TileAddr ta;
    ta.ga = xs + (int64_t)tile_I(ent) * T256 * rowbytes;
    ta.gb = xs + (int64_t)tile_J(ent) * T256 * rowbytes;
    // row of this lane inside its 8-row block (the block's first row is part
    // of the uniform base in issue_slice), and the swizzled byte column
    ta.lane_off = (uint32_t)ld_row * rowbytes + (uint32_t)ld_col;
    ta.step8 = 8u * rowbytes;
    ta.nst = (int)(rowbytes / SL);
    return ta;
}

__device__ __forceinline__ void issue_slice(const TileAddr &ta, int s, int wave, unsigned char *__restrict__ wr)
{
    unsigned char *la = wr;
    unsigned char *lb = wr + OPB;
    // uniform base of this wave's first 8-row block; block q adds q * 8 rows
    const uint32_t rowbytes = ta.step8 >> 3;
    const unsigned char *ga = ta.ga + s * SL + (uint32_t)l256::dma_row(wave, 0, 0) * rowbytes;
    const unsigned char *gb = ta.gb + s * SL + (uint32_t)l256::dma_row(wave, 0, 0) * rowbytes;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const uint32_t bq = (uint32_t)q * ta.step8;
        const int ldst = l256::dma_lds(wave, q, 0);
        __builtin_amdgcn_global_load_lds((g_void *)(ga + bq + ta.lane_off), (lds_void *)(la + ldst), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((g_void *)(gb + bq + ta.lane_off), (lds_void *)(lb + ldst), 16, 0, 0);
    }
}

// Scheduling masks of __builtin_amdgcn_sched_group_barrier.
constexpr int SG_MFMA = 0x008;
constexpr int SG_DS_READ = 0x100;

// One K slice: prefetch the following slice (or the next tile's first one)
// into the other stage, multiply this stage, then wait and synchronise.
// Within the slice the fragments of k-group g+1 are read from LDS while the
// 16 MFMAs of k-group g run (pinned with scheduling group barriers).
// The stage being read and the stage being filled arrive as restrict
// pointers: once inlined, their accesses carry distinct alias scopes, which is
// what lets the wait-count insertion see that the LDS reads below need not
// wait for the direct-to-LDS loads just issued.
template <int PREC>
__device__ __forceinline__ void slice_step_impl(typename A2<PREC>::T (&acc)[MB256][MB256], const TileAddr &cur,
                                                int s, const TileAddr &nxt, bool has_next, int wave, int wm, int wn,
                                                int lrow, int lhalf, const unsigned char *__restrict__ rd,
                                                unsigned char *__restrict__ wr)
{
    if (s + 1 < cur.nst) issue_slice(cur, s + 1, wave, wr);
    else if (has_next) issue_slice(nxt, 0, wave, wr);
    const unsigned char *la = rd;
    const unsigned char *lb = la + OPB;
    constexpr int NG = SL / 32;
    u32x4 fa[NG][MB256], fb[NG][MB256];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
        for (int m = 0; m < MB256; ++m)
            fa[g][m] = *(const u32x4 *)(la + l256::frag_lds(wm * WT256 + m * 32 + lrow, 2 * g + lhalf));
#pragma unroll
        for (int m = 0; m < MB256; ++m)
            fb[g][m] = *(const u32x4 *)(lb + l256::frag_lds(wn * WT256 + m * 32 + lrow, 2 * g + lhalf));
    }
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
        for (int a = 0; a < MB256; ++a)
#pragma unroll
            for (int b = 0; b < MB256; ++b) mma2<PREC>(acc[a][b], fa[g][a], fb[g][b]);
    // schedule: group 0 reads, then per group 16 MFMAs with the next group's
    // 8 reads spread between them (FP32 issues 4 MFMAs per fragment pair)
    constexpr int MPG = (PREC == P_F32 ? 4 : 1) * MB256 * MB256;  // MFMAs per k-group
    __builtin_amdgcn_sched_group_barrier(SG_DS_READ, 2 * MB256, 0);
#pragma unroll
    for (int g = 0; g + 1 < NG; ++g)
#pragma unroll
        for (int k = 0; k < 2 * MB256; ++k) {
            __builtin_amdgcn_sched_group_barrier(SG_MFMA, MPG / (2 * MB256), 0);
            __builtin_amdgcn_sched_group_barrier(SG_DS_READ, 1, 0);
        }
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, MPG, 0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <int PREC, int STG>
__device__ __forceinline__ void slice_step(typename A2<PREC>::T (&acc)[MB256][MB256], const TileAddr &cur, int s,
                                           const TileAddr &nxt, bool has_next, int wave, int wm, int wn, int lrow,
                                           int lhalf)
{
    slice_step_impl<PREC>(acc, cur, s, nxt, has_next, wave, wm, wn, lrow, lhalf, stage_ptr<STG>(),
                          stage_ptr<1 - STG>());
}

template <int PREC, int MODE>
__global__ __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) void screen256_kernel(ScreenArgs args)
{
    using AccT = typename A2<PREC>::T;
    using S = typename A2<PREC>::S;
    constexpr S SINF = PREC == P_I8 ? (S)0x7fffffff : (S)INFINITY;
    constexpr int ESZ = PREC == P_F32 ? 4 : (PREC == P_BF16 ? 2 : 1);

    __shared__ S sh_red[4];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = lane & 31, lhalf = lane >> 5;
    // direct-to-LDS pattern: lane i fills bytes [16 i, 16 i + 16) of a 1 KB
    // block of 8 rows, i.e. row i / 8, slot i % 8, which holds chunk slot ^ row
    const int ld_row = l256::dma_row(0, 0, lane);
    const int ld_col = l256::dma_col(lane);

    const int64_t count = (MODE & M_EMIT) ? (int64_t)*args.sel_count : args.ntiles;
    const int64_t stride = gridDim.x;

    auto next_valid = [&](int64_t t) -> int64_t {
        while (t < count && args.tiles[t] == TILE_NONE) t += stride;
        return t;
    };

    int stg = 0;
    int64_t t = next_valid(blockIdx.x);
    TileAddr cur{};
    if (t < count) {
        cur = tile_addr<ESZ>(args, args.tiles[t], wave, ld_row, ld_col);
        issue_slice(cur, 0, wave, stage_ptr<0>());
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    while (t < count) {
        const uint64_t ent = args.tiles[t];
        const uint32_t p = tile_prob(ent);
        const Prob &P = args.probs[p];
        const int64_t I = tile_I(ent), J = tile_J(ent);
        const int nst = cur.nst;
        const int64_t tn = next_valid(t + stride);
        const bool has_next = tn < count;
        const TileAddr nxt = has_next ? tile_addr<ESZ>(args, args.tiles[tn], wave, ld_row, ld_col) : cur;

        AccT acc[MB256][MB256];
#pragma unroll
        for (int a = 0; a < MB256; ++a)
#pragma unroll
            for (int b = 0; b < MB256; ++b) acc[a][b] = AccT{};

        int s = 0;
        if (stg == 1) {
            slice_step<PREC, 1>(acc, cur, s, nxt, has_next, wave, wm, wn, lrow, lhalf);
            ++s;
        }
        for (; s + 1 < nst; s += 2) {
            slice_step<PREC, 0>(acc, cur, s, nxt, has_next, wave, wm, wn, lrow, lhalf);
            slice_step<PREC, 1>(acc, cur, s + 1, nxt, has_next, wave, wm, wn, lrow, lhalf);
        }
        if (s < nst) slice_step<PREC, 0>(acc, cur, s, nxt, has_next, wave, wm, wn, lrow, lhalf);
        stg = (stg + nst) & 1;
        cur = nxt;

        // ---------------- epilogue ----------------
        // 32-bit row/column indices (n < 2^31 is enforced by the host)
        const int32_t n = (int32_t)P.n, excl = (int32_t)P.excl;
        const int32_t i0 = (int32_t)(I * T256) + wm * WT256, j0 = (int32_t)(J * T256) + wn * WT256;
        const bool full = ((int64_t)J * T256 - ((int64_t)I * T256 + T256 - 1) >= P.excl) &&
                          ((int64_t)I * T256 + T256 <= P.n) && ((int64_t)J * T256 + T256 <= P.n);
        const S *shat = (const S *)P.shat;
        S sj[MB256];
#pragma unroll
        for (int b = 0; b < MB256; ++b) sj[b] = shat[j0 + b * 32 + lrow];

        S best = SINF;
#pragma unroll
        for (int a = 0; a < MB256; ++a) {
            // rows of this lane in block a: 8*(r/4) + 4*lhalf + (r%4), four runs of 4 consecutive rows
            S si[16];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int32_t rb = i0 + a * 32 + 8 * q + 4 * lhalf;
                if constexpr (PREC == P_I8) {
                    const i32x4 v = *(const i32x4 *)(shat + rb);
                    si[4 * q] = v.x; si[4 * q + 1] = v.y; si[4 * q + 2] = v.z; si[4 * q + 3] = v.w;
                } else {
                    const f32x4 v = *(const f32x4 *)(shat + rb);
                    si[4 * q] = v.x; si[4 * q + 1] = v.y; si[4 * q + 2] = v.z; si[4 * q + 3] = v.w;
                }
            }
            if (full) {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    S m0 = part(acc[a][0][r], sj[0]);
#pragma unroll
                    for (int b = 1; b < MB256; ++b) m0 = smin(m0, part(acc[a][b][r], sj[b]));
                    best = smin(best, (S)(si[r] + m0));
                }
            } else {
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int32_t gi = i0 + a * 32 + 8 * (r >> 2) + 4 * lhalf + (r & 3);
#pragma unroll
                    for (int b = 0; b < MB256; ++b) {
                        const int32_t gj = j0 + b * 32 + lrow;
                        const bool ok = (gj - gi >= excl) && (gi < n) && (gj < n);
                        const S dv = (S)(si[r] + part(acc[a][b][r], sj[b]));
                        best = ok ? smin(best, dv) : best;
                    }
                }
            }
        }

        if constexpr (MODE & M_EMIT) {
            const double E = tile_bound(P.bmax[I], P.bmax[J], P.kpad, P.d, PREC);
            S thrU = -SINF, thrR = -SINF;
            if (args.U) {
                const double u = args.U[p];
                if constexpr (PREC == P_I8) thrU = (S)fmin(u, 2147483646.0);
                else thrU = f32_up(u + E + add_margin(u, E));
            }
            if (P.r2 >= 0.0) {
                if constexpr (PREC == P_I8) thrR = (S)fmin(floor(P.r2), 2147483646.0);
                else thrR = f32_up(P.r2 + E + add_margin(P.r2, E));
            }
            const S thr = thrU > thrR ? thrU : thrR;
            if (wmin(best) <= thr) {
#pragma unroll
                for (int a = 0; a < MB256; ++a)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int32_t gi = i0 + a * 32 + 8 * (r >> 2) + 4 * lhalf + (r & 3);
                        const S si = shat[gi];
#pragma unroll
                        for (int b = 0; b < MB256; ++b) {
                            const int32_t gj = j0 + b * 32 + lrow;
                            const S dv = (S)(si + part(acc[a][b][r], sj[b]));
                            const bool ok = full || ((gj - gi >= excl) && (gi < n) && (gj < n));
                            if (ok && dv <= thr) {
                                Cand cd;
                                cd.i = gi;
                                cd.j = gj;
                                cd.dt = (float)dv;
                                cd.p = p;
                                if (dv <= thrU) {
                                    const uint32_t idx = atomicAdd(args.cntU, 1u);
                                    if (idx < args.capU) args.candU[idx] = cd;
                                }
                                if (dv <= thrR) {
                                    const uint32_t idx = atomicAdd(args.cntR, 1u);
                                    if (idx < args.capR) args.candR[idx] = cd;
                                }
                            }
                        }
                    }
            }
        }
        if constexpr (MODE & M_MIN) {
            best = wmin(best);
            if (lane == 0) sh_red[wave] = best;
            __syncthreads();
            if (tid == 0) {
                S m = smin(smin(sh_red[0], sh_red[1]), smin(sh_red[2], sh_red[3]));
                args.tile_min[t] = __builtin_bit_cast(uint32_t, m);
            }
        }
        t = tn;
    }
}

template <int PREC>
static void launch256(int mode, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    dim3 g((unsigned)grid), b(256);
    if (mode == M_MIN) hipLaunchKernelGGL((screen256_kernel<PREC, M_MIN>), g, b, 0, st, a);
    else hipLaunchKernelGGL((screen256_kernel<PREC, M_EMIT>), g, b, 0, st, a);
}

void launch_screen256(int prec, int mode, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    if (grid <= 0) return;
    if (prec == P_F32) launch256<P_F32>(mode, a, grid, st);
    else if (prec == P_BF16) launch256<P_BF16>(mode, a, grid, st);
    else launch256<P_I8>(mode, a, grid, st);
}

}  // namespace cpmi
