// Persistent 256x256 Gram screen for CDNA4 (gfx950).
//
// Same contract as the 128-tile screen in screen.hip (tile minimum of the
// screen value D~ = s^_i + s^_j - 2 <x~_i, x~_j>, radius and threshold
// emission), organised for throughput on large problems:
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

template <int PREC, int MODE>
__global__ __launch_bounds__(256, 1) void screen256_kernel(ScreenArgs args)
{
    using AccT = typename A2<PREC>::T;
    using S = typename A2<PREC>::S;
    constexpr S SINF = PREC == P_I8 ? (S)0x7fffffff : (S)INFINITY;
    constexpr int ESZ = PREC == P_F32 ? 4 : (PREC == P_BF16 ? 2 : 1);

    __shared__ __attribute__((aligned(1024))) unsigned char lds[4 * OPB];  // [stage][A | B]
    __shared__ S sh_red[4];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = lane & 31, lhalf = lane >> 5;
    // direct-to-LDS pattern: lane i fills bytes [16 i, 16 i + 16) of a 1 KB
    // block of 8 rows, i.e. row i / 8, slot i % 8, which holds chunk slot ^ row
    const int ld_row = lane >> 3;
    const int ld_col = ((lane & 7) ^ ld_row) << 4;

    const int64_t count = (MODE & M_EMIT_U) ? (int64_t)*args.sel_count : args.ntiles;
    const int64_t stride = gridDim.x;

    auto next_valid = [&](int64_t t) -> int64_t {
        while (t < count && args.tiles[t] == TILE_NONE) t += stride;
        return t;
    };
    // issue the loads of K slice `s` of tile entry `ent` into LDS stage `stg`
    auto issue = [&](uint64_t ent, int s, int stg) {
        const Prob &P = args.probs[tile_prob(ent)];
        const int64_t rowbytes = (int64_t)P.kpad * ESZ;
        const unsigned char *xs = (const unsigned char *)P.xs;
        const unsigned char *ga = xs + (int64_t)tile_I(ent) * T256 * rowbytes + (int64_t)s * SL + ld_col;
        const unsigned char *gb = xs + (int64_t)tile_J(ent) * T256 * rowbytes + (int64_t)s * SL + ld_col;
        unsigned char *la = lds + stg * 2 * OPB;
        unsigned char *lb = la + OPB;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int R0 = (wave * 8 + q) * 8;
            const int64_t row = R0 + ld_row;
            __builtin_amdgcn_global_load_lds((g_void *)(ga + row * rowbytes), (lds_void *)(la + R0 * SL), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((g_void *)(gb + row * rowbytes), (lds_void *)(lb + R0 * SL), 16, 0, 0);
        }
    };

    int stg = 0;
    int64_t t = next_valid(blockIdx.x);
    if (t < count) issue(args.tiles[t], 0, stg);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();

    while (t < count) {
        const uint64_t ent = args.tiles[t];
        const uint32_t p = tile_prob(ent);
        const Prob &P = args.probs[p];
        const int64_t I = tile_I(ent), J = tile_J(ent);
        const int nst = (int)((int64_t)P.kpad * ESZ / SL);
        const int64_t tn = next_valid(t + stride);

        AccT acc[MB256][MB256];
#pragma unroll
        for (int a = 0; a < MB256; ++a)
#pragma unroll
            for (int b = 0; b < MB256; ++b) acc[a][b] = AccT{};

        for (int s = 0; s < nst; ++s) {
            if (s + 1 < nst) issue(ent, s + 1, stg ^ 1);
            else if (tn < count) issue(args.tiles[tn], 0, stg ^ 1);
            const unsigned char *la = lds + stg * 2 * OPB;
            const unsigned char *lb = la + OPB;
#pragma unroll
            for (int g = 0; g < SL / 32; ++g) {
                const int sw = (((2 * g + lhalf) ^ (lrow & 7)) << 4);
                u32x4 fa[MB256], fb[MB256];
#pragma unroll
                for (int m = 0; m < MB256; ++m)
                    fa[m] = *(const u32x4 *)(la + (wm * WT256 + m * 32 + lrow) * SL + sw);
#pragma unroll
                for (int m = 0; m < MB256; ++m)
                    fb[m] = *(const u32x4 *)(lb + (wn * WT256 + m * 32 + lrow) * SL + sw);
#pragma unroll
                for (int a = 0; a < MB256; ++a)
#pragma unroll
                    for (int b = 0; b < MB256; ++b) mma2<PREC>(acc[a][b], fa[a], fb[b]);
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            stg ^= 1;
        }

        // ---------------- epilogue ----------------
        const int64_t n = P.n, excl = P.excl;
        const int64_t i0 = I * T256 + wm * WT256, j0 = J * T256 + wn * WT256;
        const bool full = (J * T256 - (I * T256 + T256 - 1) >= excl) && (I * T256 + T256 <= n) && (J * T256 + T256 <= n);
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
                const int64_t rb = i0 + a * 32 + 8 * q + 4 * lhalf;
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
                    const int64_t gi = i0 + a * 32 + 8 * (r >> 2) + 4 * lhalf + (r & 3);
#pragma unroll
                    for (int b = 0; b < MB256; ++b) {
                        const int64_t gj = j0 + b * 32 + lrow;
                        const bool ok = (gj - gi >= excl) && (gi < n) && (gj < n);
                        const S dv = (S)(si[r] + part(acc[a][b][r], sj[b]));
                        best = ok ? smin(best, dv) : best;
                    }
                }
            }
        }

        if constexpr (MODE & (M_EMIT_R | M_EMIT_U)) {
            const double E = tile_bound(P.bmax[I], P.bmax[J], P.kpad, P.d, PREC);
            S thr;
            if constexpr (MODE & M_EMIT_U) {
                const double u = args.U[p];
                if constexpr (PREC == P_I8) thr = (S)fmin(u, 2147483646.0);
                else thr = f32_up(u + E + add_margin(u, E));
            } else {
                if constexpr (PREC == P_I8) thr = (S)fmin(floor(P.r2), 2147483646.0);
                else thr = f32_up(P.r2 + E + add_margin(P.r2, E));
            }
            if (wmin(best) <= thr) {
                Cand *cand = (MODE & M_EMIT_U) ? args.candU : args.candR;
                uint32_t *cnt = (MODE & M_EMIT_U) ? args.cntU : args.cntR;
                const uint32_t cap = (MODE & M_EMIT_U) ? args.capU : args.capR;
#pragma unroll
                for (int a = 0; a < MB256; ++a)
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int64_t gi = i0 + a * 32 + 8 * (r >> 2) + 4 * lhalf + (r & 3);
                        const S si = shat[gi];
#pragma unroll
                        for (int b = 0; b < MB256; ++b) {
                            const int64_t gj = j0 + b * 32 + lrow;
                            const S dv = (S)(si + part(acc[a][b][r], sj[b]));
                            const bool ok = full || ((gj - gi >= excl) && (gi < n) && (gj < n));
                            if (ok && dv <= thr) {
                                const uint32_t idx = atomicAdd(cnt, 1u);
                                if (idx < cap) {
                                    Cand cd;
                                    cd.i = (int32_t)gi;
                                    cd.j = (int32_t)gj;
                                    cd.dt = (float)dv;
                                    cd.p = p;
                                    cand[idx] = cd;
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
    switch (mode) {
    case M_MIN: hipLaunchKernelGGL((screen256_kernel<PREC, M_MIN>), g, b, 0, st, a); break;
    case M_MIN | M_EMIT_R: hipLaunchKernelGGL((screen256_kernel<PREC, M_MIN | M_EMIT_R>), g, b, 0, st, a); break;
    case M_EMIT_U: hipLaunchKernelGGL((screen256_kernel<PREC, M_EMIT_U>), g, b, 0, st, a); break;
    default: break;
    }
}

void launch_screen256(int prec, int mode, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    if (grid <= 0) return;
    if (prec == P_F32) launch256<P_F32>(mode, a, grid, st);
    else if (prec == P_BF16) launch256<P_BF16>(mode, a, grid, st);
    else launch256<P_I8>(mode, a, grid, st);
}

}  // namespace cpmi
