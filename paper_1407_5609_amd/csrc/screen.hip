// Gram-form pair screen on the CDNA4 matrix cores, with a fused epilogue.
//
// The paper's hot loop evaluates d(p_i, p_j) for the surviving pairs and keeps
// the least one (MPR step 5, Section 3.3) or emits the pair when d <= R
// (MPR-FRNNS step 5, Section 3.5); brute force does this for every pair in
// O(n^2 l) (Section 3). Here every admissible pair of a tile is screened at
// once: D~_ij = s^_i + s^_j - 2 <x~_i, x~_j>, the inner products coming from
// MFMA tiles (FP32, BF16 or INT8 operands), then
//   - M_MIN:  the tile minimum of D~ is recorded (one word per tile);
//   - M_EMIT: (second pass, on the tiles whose lower bound reaches U or R^2)
//             pairs with D~ <= U + E_tile are appended to the closest-pair
//             candidates (U the proven upper bound of the minimum) and pairs
//             with D~ <= R^2 + E_tile to the radius candidates.
// E_tile is the rigorous screening-error bound of bound.h, so every pair that
// can be the minimum or lie within the radius reaches the FP64 verifier.
//
// Tiling: a work-group of 256 threads (4 wave64s in a 2x2 grid) owns a TILE x
// TILE block of the pair matrix; each wave owns (TILE/2)^2 outputs as 32x32
// MFMA blocks. K is streamed through LDS in 128-byte row slices (FP32: 32,
// BF16: 64, INT8: 128 elements), with the next slice's global loads in flight
// while the current one is multiplied. LDS rows are padded to 144 bytes so
// that the 16-byte fragment reads of 32 consecutive rows do not collide.
#include "bound.h"
#include "cpmi_internal.h"

namespace cpmi {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const u32x4 gu32x4;  // global-memory view

constexpr int NTHREADS = 256;
constexpr int SLICE = 128;       // bytes of K per row per LDS stage
constexpr int LSTRIDE = 144;     // LDS row stride in bytes

template <int PREC> struct Acc { using T = f32x16; using S = float; };
template <> struct Acc<P_I8> { using T = i32x16; using S = int; };

// One 16-byte fragment per lane covers 32 bytes of K across the two lane
// halves: lane l holds row (l % 32), bytes [(l/32)*16, (l/32)*16 + 16). The
// same K placement is used for both operands, so the products pair up equal
// coordinates whatever order the hardware reduces them in.
template <int PREC>
__device__ __forceinline__ void mma(typename Acc<PREC>::T &c, const u32x4 &a, const u32x4 &b)
{
    if constexpr (PREC == P_F32) {
        // 4 floats per lane = 4 consecutive K-steps of the 32x32x2 FP32 MFMA
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

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

template <int PREC, int TILE, int MODE>
__global__ __launch_bounds__(NTHREADS) void screen_kernel(ScreenArgs args)
{
    using AccT = typename Acc<PREC>::T;
    using S = typename Acc<PREC>::S;
    constexpr int WT = TILE / 2;                 // wave tile edge
    constexpr int MB = WT / 32;                  // MFMA blocks per wave edge
    constexpr int CPT = TILE * (SLICE / 16) / NTHREADS;  // 16-byte chunks per thread per operand
    constexpr S SINF = PREC == P_I8 ? (S)0x7fffffff : (S)INFINITY;

    __shared__ __attribute__((aligned(16))) unsigned char lds[2 * TILE * LSTRIDE];
    __shared__ S sh_si[TILE];
    __shared__ S sh_sj[TILE];

    unsigned char *ldsA = lds;
    unsigned char *ldsB = lds + TILE * LSTRIDE;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lrow = lane & 31, lhalf = lane >> 5;

    const bool dense = (MODE & M_EMIT) && args.sel_dense && (int64_t)*args.sel_count * 4 > args.ntiles;
    const int64_t count = (MODE & M_EMIT) && !dense ? (int64_t)*args.sel_count : args.ntiles;
    const uint64_t *list = dense ? args.sel_dense : args.tiles;

    for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
        const uint64_t ent = list[t];
        if (ent == TILE_NONE) continue;
        const uint32_t p = tile_prob(ent);
        const int64_t I = tile_I(ent), J = tile_J(ent);
        const Prob &P = args.probs[p];
        const int64_t rowbytes = (int64_t)P.kpad * (PREC == P_F32 ? 4 : (PREC == P_BF16 ? 2 : 1));
        const unsigned char *ga = (const unsigned char *)P.xs + I * TILE * rowbytes;
        const unsigned char *gb = (const unsigned char *)P.xs + J * TILE * rowbytes;
        const int nst = (int)(rowbytes / SLICE);
        const S *shat = (const S *)P.shat;

        // stage the row scalars of both blocks
        for (int q = tid; q < TILE; q += NTHREADS) {
            sh_si[q] = shat[I * TILE + q];
            sh_sj[q] = shat[J * TILE + q];
        }

        AccT acc[MB][MB];
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int b = 0; b < MB; ++b) acc[a][b] = AccT{};

        u32x4 ra[CPT], rb[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int c = tid + q * NTHREADS;
            const int row = c >> 3, col = (c & 7) * 16;
            ra[q] = *(gu32x4 *)(ga + row * rowbytes + col);
            rb[q] = *(gu32x4 *)(gb + row * rowbytes + col);
        }

        for (int s = 0; s < nst; ++s) {
            __syncthreads();
#pragma unroll
            for (int q = 0; q < CPT; ++q) {
                const int c = tid + q * NTHREADS;
                const int row = c >> 3, col = (c & 7) * 16;
                *(u32x4 *)(ldsA + row * LSTRIDE + col) = ra[q];
                *(u32x4 *)(ldsB + row * LSTRIDE + col) = rb[q];
            }
            __syncthreads();
            {
                // next slice (the last iteration re-reads its own slice: the
                // loads stay unconditional so the staging registers are never
                // demoted to scratch memory)
                const int64_t off = (int64_t)(s + 1 < nst ? s + 1 : s) * SLICE;
#pragma unroll
                for (int q = 0; q < CPT; ++q) {
                    const int c = tid + q * NTHREADS;
                    const int row = c >> 3, col = (c & 7) * 16;
                    ra[q] = *(gu32x4 *)(ga + row * rowbytes + off + col);
                    rb[q] = *(gu32x4 *)(gb + row * rowbytes + off + col);
                }
            }
#pragma unroll
            for (int g = 0; g < SLICE / 32; ++g) {
                u32x4 fa[MB], fb[MB];
#pragma unroll
                for (int m = 0; m < MB; ++m)
                    fa[m] = *(const u32x4 *)(ldsA + (wm * WT + m * 32 + lrow) * LSTRIDE + g * 32 + lhalf * 16);
#pragma unroll
                for (int m = 0; m < MB; ++m)
                    fb[m] = *(const u32x4 *)(ldsB + (wn * WT + m * 32 + lrow) * LSTRIDE + g * 32 + lhalf * 16);
#pragma unroll
                for (int a = 0; a < MB; ++a)
#pragma unroll
                    for (int b = 0; b < MB; ++b) mma<PREC>(acc[a][b], fa[a], fb[b]);
            }
        }

        // ---------------- epilogue ----------------
        const int64_t n = P.n;
        const int64_t excl = P.excl;
        const int64_t i0 = I * TILE, j0 = J * TILE;
        // every pair of the tile admissible? (min j - max i >= excl, all rows real)
        const bool full = (j0 - (i0 + TILE - 1) >= excl) && (i0 + TILE <= n) && (j0 + TILE <= n);
        const double E = tile_bound(P.bmax[I], P.bmax[J], P.kpad, P.d, PREC, SCREEN_EPILOGUE);
        S thrU = -SINF, thrR = -SINF, thrIn = -SINF;
        if constexpr (MODE & M_EMIT) {
            if (args.U) {
                const double u = args.U[p];
                if constexpr (PREC == P_I8) thrU = (S)fmin(u, 2147483646.0);
                else thrU = f32_up(u + E + add_margin(u, E));
            }
            if (P.r2 >= 0.0) {
                if constexpr (PREC == P_I8) thrR = (S)fmin(floor(P.r2), 2147483646.0);
                else thrR = f32_up(P.r2 + E + add_margin(P.r2, E));
                if (args.cntIn) {
                    if constexpr (PREC == P_I8) thrIn = thrR;   // exact: no band
                    else thrIn = f32_down(P.r2 - E - add_margin(P.r2, E));
                }
            }
        }
        // every element of this lane: (row, column, screen value, admissible)
        auto each = [&](auto f) {
#pragma unroll
            for (int b = 0; b < MB; ++b) {
                const int jl = wn * WT + b * 32 + lrow;
                const S sj = sh_sj[jl];
                const int64_t gj = j0 + jl;
#pragma unroll
                for (int a = 0; a < MB; ++a) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) {
                        const int il = wm * WT + a * 32 + 8 * (r >> 2) + 4 * lhalf + (r & 3);
                        const int64_t gi = i0 + il;
                        S dv;
                        if constexpr (PREC == P_I8)
                            dv = sh_si[il] + (sj - 2 * acc[a][b][r]);
                        else
                            dv = sh_si[il] + fmaf(-2.0f, acc[a][b][r], sj);
                        const bool ok = full || ((gj - gi >= excl) && (gi < n) && (gj < n));
                        f(gi, gj, dv, ok);
                    }
                }
            }
        };
        if constexpr (MODE & M_DUMP) {
            S *out = (S *)args.dump + (size_t)t * (TILE * TILE);
            each([&](int64_t gi, int64_t gj, S dv, bool) { out[(gi - i0) * TILE + (gj - j0)] = dv; });
        }
        S mn = SINF;
        if constexpr (MODE & M_MIN) {
            each([&](int64_t, int64_t, S dv, bool ok) {
                dv = ok ? dv : SINF;
                mn = PREC == P_I8 ? (S)min((int)mn, (int)dv) : (S)fminf(mn, dv);
            });
        }
        if constexpr (MODE & M_EMIT) {
            // count this lane's pairs, reserve them with one atomic per wave
            // and counter, then write them
            uint32_t nU = 0, nR = 0, nIn = 0;
            each([&](int64_t, int64_t, S dv, bool ok) {
                nU += ok & (dv <= thrU);
                const bool in = ok & (dv <= thrIn);
                nIn += in;
                nR += ok & !in & (dv <= thrR);
            });
            if (args.cntIn) wave_count(args.cntIn, nIn);
            uint64_t kU = wave_reserve(args.cntU, nU), kR = wave_reserve(args.cntR, nR);
            if (__any(nU + nR != 0)) {
                each([&](int64_t gi, int64_t gj, S dv, bool ok) {
                    Cand cd;
                    cd.i = (int32_t)gi;
                    cd.j = (int32_t)gj;
                    cd.dt = (float)dv;
                    cd.p = p;
                    if (ok & (dv <= thrU)) {
                        if (kU < args.capU) args.candU[kU] = cd;
                        ++kU;
                    }
                    if (ok & !(dv <= thrIn) & (dv <= thrR)) {
                        if (kR < args.capR) args.candR[kR] = cd;
                        ++kR;
                    }
                });
            }
        }
        if constexpr (MODE & M_MIN) {
            // each wave stores the minimum of its quarter of the tile
            mn = wave_min(mn);
            if (lane == 0) args.tile_min[4 * t + wave] = __builtin_bit_cast(uint32_t, mn);
        }
        __syncthreads();  // LDS (sh_si/sh_sj) is reused by the next tile
    }
}

template <int PREC, int TILE>
static void launch_t(int mode, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    dim3 g((unsigned)grid), b(NTHREADS);
    if (mode == M_MIN) hipLaunchKernelGGL((screen_kernel<PREC, TILE, M_MIN>), g, b, 0, st, a);
    else if (mode == M_DUMP) hipLaunchKernelGGL((screen_kernel<PREC, TILE, M_DUMP>), g, b, 0, st, a);
    else hipLaunchKernelGGL((screen_kernel<PREC, TILE, M_EMIT>), g, b, 0, st, a);
}

void launch_screen256(int prec, int mode, bool masked, const ScreenArgs &a, int64_t grid, hipStream_t st);

void launch_screen(int prec, int tile, int mode, bool masked, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    if (grid <= 0) return;
    if (tile == 256) {
        launch_screen256(prec, mode, masked, a, grid, st);
    } else {
        if (prec == P_F32) launch_t<P_F32, 128>(mode, a, grid, st);
        else if (prec == P_BF16) launch_t<P_BF16, 128>(mode, a, grid, st);
        else launch_t<P_I8, 128>(mode, a, grid, st);
    }
}

// ---------------------------------------------------------------------------
// Debug: one 32x32 MFMA block through the same fragment path, to check the
// operand and accumulator lane layouts on the device. A and B are 32 rows of
// 32 bytes (K slice), C receives the 32x32 result (as float; int8 converted).
// ---------------------------------------------------------------------------
template <int PREC>
__global__ void mfma_probe_kernel(const unsigned char *A, const unsigned char *B, float *C)
{
    using AccT = typename Acc<PREC>::T;
    const int lane = threadIdx.x;
    const int lrow = lane & 31, lhalf = lane >> 5;
    const u32x4 a = *(const u32x4 *)(A + lrow * 32 + lhalf * 16);
    const u32x4 b = *(const u32x4 *)(B + lrow * 32 + lhalf * 16);
    AccT acc = AccT{};
    mma<PREC>(acc, a, b);
    for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * lhalf + (r & 3);
        C[row * 32 + lrow] = (float)acc[r];
    }
}

// Sustained matrix-core rate: every wave keeps 16 independent accumulations
// (the screen's instruction and register budget: 256 accumulator registers)
// busy for `iters` rounds with operands held in registers, so no memory
// traffic limits it; one store per lane at the end keeps the work alive.
template <int PREC>
__global__ __launch_bounds__(256, 1) void mfma_peak_kernel(int iters, float *out)
{
    using AccT = typename Acc<PREC>::T;
    const int lane = threadIdx.x & 63;
    // small non-zero operands (varying by lane) that keep the sums finite
    const uint32_t pat = PREC == P_I8 ? 0x01020301u * (uint32_t)(1 + (lane & 3))
                                      : (PREC == P_BF16 ? 0x3a003a00u + (uint32_t)lane * 0x00010001u
                                                        : 0x3a000000u + (uint32_t)lane);
    const u32x4 a = {pat, pat ^ 0x00100010u, pat, pat ^ 0x00200020u};
    const u32x4 b0 = {pat ^ 0x00300030u, pat, pat ^ 0x00100010u, pat};
    const u32x4 b1 = {pat, pat ^ 0x00200020u, pat, pat ^ 0x00300030u};
    AccT acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = AccT{};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 16; ++q) mma<PREC>(acc[q], a, (q & 1) ? b1 : b0);
    }
    float sum = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q)
#pragma unroll
        for (int r = 0; r < 16; ++r) sum += (float)acc[q][r];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

void launch_mfma_peak(int prec, int iters, int grid, float *out, hipStream_t st)
{
    if (prec == P_F32) hipLaunchKernelGGL(mfma_peak_kernel<P_F32>, dim3(grid), dim3(256), 0, st, iters, out);
    else if (prec == P_BF16) hipLaunchKernelGGL(mfma_peak_kernel<P_BF16>, dim3(grid), dim3(256), 0, st, iters, out);
    else hipLaunchKernelGGL(mfma_peak_kernel<P_I8>, dim3(grid), dim3(256), 0, st, iters, out);
}

void launch_mfma_probe(int prec, const void *A, const void *B, float *C, hipStream_t st)
{
    const unsigned char *a = (const unsigned char *)A, *b = (const unsigned char *)B;
    if (prec == P_F32) hipLaunchKernelGGL(mfma_probe_kernel<P_F32>, dim3(1), dim3(64), 0, st, a, b, C);
    else if (prec == P_BF16) hipLaunchKernelGGL(mfma_probe_kernel<P_BF16>, dim3(1), dim3(64), 0, st, a, b, C);
    else hipLaunchKernelGGL(mfma_probe_kernel<P_I8>, dim3(1), dim3(64), 0, st, a, b, C);
}

}  // namespace cpmi
