// Persistent 256x256 Gram screen for CDNA4 (gfx950).
//
// Same contract as the 128-tile screen in screen.hip (pass 1: tile minimum of
// the screen value D~ = s^_i + s^_j - 2 <x~_i, x~_j>; pass 2: emission of the
// pairs within the closest-pair or radius thresholds), organised for
// throughput on large problems:
//   * a persistent grid walks the tile list with stride gridDim.x, so a
//     work-group keeps the slots of one XCD chunk of the list;
//   * K slices (64 bytes per row) go straight from global memory into LDS
//     with global_load_lds_dwordx4 (no staging registers) through a ring of
//     four stages: the loads run three slices ahead of the multiply, across
//     tile boundaries, with one barrier per slice (rows of 4k + 2 slices: the
//     K2 form, whose tiles start at stage 0 or 2);
//   * each 16-row, 1 KB LDS block stores row r's 16-byte chunk c at slot
//     c ^ ((r >> 2) & 3), so the fragment reads of 16 consecutive rows hit
//     all 64 banks once (layout256.h);
//   * 4 waves in a 2x2 grid, each owning 128x128 outputs as 4x4 32x32 MFMA
//     blocks (256 accumulators per lane);
//   * FP32 and BF16: the row scalars are folded into the product (one extra
//     matrix-core step per block starts the accumulators at
//     -(s^_i + s^_j)/2), so the screen value is -2 acc and the tile minimum
//     is -2 times the largest accumulator (half a max3 per element, no
//     per-element arithmetic). INT8: s^_i + (s^_j - 2 G) in exact int32;
//   * emission (pass 2) runs only when the wave's minimum is within a
//     threshold: each lane counts its pairs, one atomic add per wave and
//     counter reserves their slots, and a second scan writes them.
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
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void g_void;
// Read-only kernel inputs (tile list, problem descriptors) are read through
// the constant address space: with uniform addresses that gives scalar loads,
// which are counted apart from the vector loads and so never wait behind the
// direct-to-LDS loads in flight.
typedef __attribute__((address_space(4))) const uint64_t c_u64;
typedef __attribute__((address_space(4))) const Prob c_prob;

namespace {

constexpr int T256 = 256;         // tile edge
constexpr int WT256 = 128;        // wave tile edge
constexpr int MB256 = 4;          // 32x32 blocks per wave edge
constexpr int SL = l256::SLICE;   // K slice, bytes per row (64)
constexpr int OPB = T256 * SL;    // one operand slice in LDS (16 KB)

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

// This lane's index, recomputed by the hardware at each use: values derived
// from a lane index computed once would otherwise stay live (and be spilled)
// across the register-hungry epilogue, and their reloads would wait behind the
// loads in flight.
__device__ __forceinline__ int fresh_lane()
{
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// 4 x this lane's index as a 64-bit value, both halves written by the
// hardware at each use (so that no widened lane value is kept across loops).
__device__ __forceinline__ uint64_t fresh_lane_bytes4()
{
    uint32_t lo, hi;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0\n\t"
                 "v_lshlrev_b32 %0, 2, %0\n\tv_mov_b32 %1, 0"
                 : "=&v"(lo), "=v"(hi));
    return (uint64_t)hi << 32 | lo;
}

// Minimum over the wave, returned in every lane: within each row of 16 lanes
// by DPP steps (lane pairs, then quad pairs, then row-half and row mirrors:
// every lane ends with its row's minimum), then the four rows through
// lanes 0, 16, 32 and 48. No LDS round trip, no lane index.
template <int CTRL, typename S> __device__ __forceinline__ S dpp_min(S v)
{
    return smin(v, __builtin_bit_cast(S, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf,
                                                                     false)));
}
template <typename S> __device__ __forceinline__ S wmin(S v)
{
    v = dpp_min<0xb1>(v);    // quad_perm [1,0,3,2]
    v = dpp_min<0x4e>(v);    // quad_perm [2,3,0,1]
    v = dpp_min<0x141>(v);   // row_half_mirror
    v = dpp_min<0x140>(v);   // row_mirror
    const S a = __builtin_bit_cast(S, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
    const S b = __builtin_bit_cast(S, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
    const S c = __builtin_bit_cast(S, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
    const S d = __builtin_bit_cast(S, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
    return smin(smin(a, b), smin(c, d));
}

// s^_j - 2 g  (float: one fma; int8: exact int32)
[[maybe_unused]] __device__ __forceinline__ float part(float g, float sj) { return fmaf(-2.0f, g, sj); }
__device__ __forceinline__ int part(int g, int sj) { return sj - 2 * g; }

// Bits of one 32-bit lane value as S. (Taken through a scalar argument: the
// compiler lowers a bit cast of a vector element such as v.y as a read of the
// vector's first element.)
template <typename S> __device__ __forceinline__ S bits_as(uint32_t u) { return __builtin_bit_cast(S, u); }

// Reads of the per-tile row scalars, which direct-to-LDS loads wrote. Those
// loads are older than every K slice of the tile, so the per-slice load waits
// and barriers have already made them visible; the compiler cannot see that
// and would drain every load in flight (including the next tile's slices)
// before a plain read. These reads wait for themselves, in the same asm block.
// Four 16-byte values at p, p + 32 B, p + 64 B, p + 96 B.
__device__ __forceinline__ void lds_landed_4x128(const void *p, u32x4 &a, u32x4 &b, u32x4 &c, u32x4 &d)
{
    const uint32_t ad = (uint32_t)(uintptr_t)p;
    asm volatile("ds_read_b128 %0, %4\n\t"
                 "ds_read_b128 %1, %4 offset:32\n\t"
                 "ds_read_b128 %2, %4 offset:64\n\t"
                 "ds_read_b128 %3, %4 offset:96\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(a), "=&v"(b), "=&v"(c), "=&v"(d)
                 : "v"(ad));
}
// Four 4-byte values at p, p + 128 B, p + 256 B, p + 384 B.
__device__ __forceinline__ u32x4 lds_landed_4x32(const void *p)
{
    u32x2 lo, hi;
    const uint32_t a = (uint32_t)(uintptr_t)p;
    asm volatile("ds_read2_b32 %0, %2 offset1:32\n\t"
                 "ds_read2_b32 %1, %2 offset0:64 offset1:96\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(lo), "=&v"(hi)
                 : "v"(a));
    return u32x4{lo.x, lo.y, hi.x, hi.y};
}

// Four 8-byte values at p, p + 256 B, p + 512 B, p + 768 B, as (first two,
// last two).
__device__ __forceinline__ void lds_landed_4x64(const void *p, u32x4 &lo, u32x4 &hi)
{
    const uint32_t a = (uint32_t)(uintptr_t)p;
    asm volatile("ds_read2_b64 %0, %2 offset1:32\n\t"
                 "ds_read2_b64 %1, %2 offset0:64 offset1:96\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(lo), "=&v"(hi)
                 : "v"(a));
}

}  // namespace

// The four LDS stages are distinct __shared__ objects and every slice step
// names its stages at compile time, so the compiler can see that the
// direct-to-LDS loads into one stage never alias the fragment reads of
// another and does not make those reads wait for the loads in flight.
__shared__ __attribute__((aligned(1024))) unsigned char g_stage0[2 * OPB];
__shared__ __attribute__((aligned(1024))) unsigned char g_stage1[2 * OPB];
__shared__ __attribute__((aligned(1024))) unsigned char g_stage2[2 * OPB];
__shared__ __attribute__((aligned(1024))) unsigned char g_stage3[2 * OPB];

template <int STG> __device__ __forceinline__ unsigned char *stage_ptr()
{
    return STG == 0 ? g_stage0 : (STG == 1 ? g_stage1 : (STG == 2 ? g_stage2 : g_stage3));
}

// Per-tile addressing of the direct-to-LDS loads: uniform values only (a
// base per operand), so the load cursor lives in scalar registers; the
// per-lane offset is recomputed at each issue from a fresh lane index.
struct TileAddr {
    const unsigned char *ga;  // operand A rows of the tile
    const unsigned char *gb;  // operand B rows of the tile
    uint32_t rowbytes;
    int nst;                  // K slices of the tile
};

template <int ESZ>
__device__ __forceinline__ TileAddr tile_addr(const ScreenArgs &args, uint64_t ent)
{
    const c_prob &P = ((c_prob *)args.probs)[tile_prob(ent)];
    const uint32_t rowbytes = (uint32_t)P.kpad * ESZ;
    const unsigned char *xs = (const unsigned char *)P.xs;
    TileAddr ta;
    // start of the 256-row blocks I and J (the same in either layout)
    ta.ga = xs + (int64_t)tile_I(ent) * T256 * rowbytes;
    ta.gb = xs + (int64_t)tile_J(ent) * T256 * rowbytes;
    ta.rowbytes = rowbytes;
    ta.nst = (int)(rowbytes / SL);
    return ta;
}

// The 8 direct-to-LDS loads of one wave for K slice s of a tile (4 blocks of
// 16 rows per operand). The operand is slice-major per 256-row block
// (layout256.h: xs_offset), so slice s of the tile's rows is 16 KB of
// consecutive memory and each load reads 1 KB of it. The wave's four blocks
// lie 1 KB apart both in memory and in the stage, so they share one address
// pair and differ in the instruction offset, which the hardware adds to the
// global and to the LDS address alike.
__device__ __forceinline__ void issue_slice(const TileAddr &ta, int s, int wave, unsigned char *__restrict__ wr)
{
    static_assert(l256::dma_lds(0, 1, 0) - l256::dma_lds(0, 0, 0) == 1024 &&
                      (l256::dma_row(0, 1, 0) - l256::dma_row(0, 0, 0)) * SL == 1024 && l256::NQ == 4,
                  "a wave's four blocks lie 1 KB apart in the stage and in the operand");
    unsigned char *la = wr;
    unsigned char *lb = wr + OPB;
    // (row within a 16-row block) * SL + swizzled column; the column swizzle
    // of a lane does not depend on the block (layout256.h)
    const int lane = fresh_lane();
    const uint32_t lane_off = (uint32_t)l256::dma_row(0, 0, lane) * SL + (uint32_t)l256::dma_col(0, 0, lane);
    const uint32_t rb = (uint32_t)s * (T256 * SL) + (uint32_t)l256::dma_row(wave, 0, 0) * SL;
    const int ldst = l256::dma_lds(wave, 0, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.ga + rb + lane_off), (lds_void *)(la + ldst), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.ga + rb + lane_off), (lds_void *)(la + ldst), 16, 1024, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.ga + rb + lane_off), (lds_void *)(la + ldst), 16, 2048, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.ga + rb + lane_off), (lds_void *)(la + ldst), 16, 3072, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.gb + rb + lane_off), (lds_void *)(lb + ldst), 16, 0, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.gb + rb + lane_off), (lds_void *)(lb + ldst), 16, 1024, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.gb + rb + lane_off), (lds_void *)(lb + ldst), 16, 2048, 0);
    __builtin_amdgcn_global_load_lds((g_void *)(ta.gb + rb + lane_off), (lds_void *)(lb + ldst), 16, 3072, 0);
}

// Scheduling masks of __builtin_amdgcn_sched_group_barrier.
constexpr int SG_MFMA = 0x008;
constexpr int SG_VMEM_READ = 0x020;
constexpr int SG_DS_READ = 0x100;

// s_waitcnt immediates (gfx9 encoding: vmcnt[3:0] | expcnt << 4 | lgkmcnt << 8 | vmcnt[5:4] << 14).
// WAIT_SLICE: at most the 16 loads of the two newest slices in flight, all LDS reads done.
constexpr int WAIT_SLICE = (16 & 15) | (7 << 4) | (0 << 8) | ((16 >> 4) << 14);

template <int PREC> using Frags = u32x4[MB256];

template <int PREC>
__device__ __forceinline__ void read_group(Frags<PREC> &fa, Frags<PREC> &fb, const unsigned char *__restrict__ st,
                                           int g, int wm, int wn, int lrow, int lhalf)
{
#pragma unroll
    for (int m = 0; m < MB256; ++m)
        fa[m] = *(const u32x4 *)(st + l256::frag_lds(wm * WT256 + m * 32 + lrow, 2 * g + lhalf));
#pragma unroll
    for (int m = 0; m < MB256; ++m)
        fb[m] = *(const u32x4 *)(st + OPB + l256::frag_lds(wn * WT256 + m * 32 + lrow, 2 * g + lhalf));
}

// k-group g of a stage, as read_group, through reads the compiler does not
// track (they wait for themselves, in the same asm block): for a stage that
// has landed on every path that reaches the read, where the compiler cannot
// see that. Rows 32 apart share their slot swizzle, so the four blocks of an
// operand sit 2 KB apart from one address.
template <int PREC>
__device__ __forceinline__ void read_group_landed(Frags<PREC> &fa, Frags<PREC> &fb, const unsigned char *st, int g,
                                                  int wm, int wn, int lrow, int lhalf)
{
    const uint32_t pa = (uint32_t)(uintptr_t)(st + l256::frag_lds(wm * WT256 + lrow, 2 * g + lhalf));
    const uint32_t pb = (uint32_t)(uintptr_t)(st + OPB + l256::frag_lds(wn * WT256 + lrow, 2 * g + lhalf));
    asm volatile("ds_read_b128 %0, %8\n\t"
                 "ds_read_b128 %1, %8 offset:2048\n\t"
                 "ds_read_b128 %2, %8 offset:4096\n\t"
                 "ds_read_b128 %3, %8 offset:6144\n\t"
                 "ds_read_b128 %4, %9\n\t"
                 "ds_read_b128 %5, %9 offset:2048\n\t"
                 "ds_read_b128 %6, %9 offset:4096\n\t"
                 "ds_read_b128 %7, %9 offset:6144\n\t"
                 "s_waitcnt lgkmcnt(0)"
                 : "=&v"(fa[0]), "=&v"(fa[1]), "=&v"(fa[2]), "=&v"(fa[3]), "=&v"(fb[0]), "=&v"(fb[1]), "=&v"(fb[2]),
                   "=&v"(fb[3])
                 : "v"(pa), "v"(pb));
}

template <int PREC>
__device__ __forceinline__ void mma_group(typename A2<PREC>::T (&acc)[MB256][MB256], const Frags<PREC> &fa,
                                          const Frags<PREC> &fb)
{
#pragma unroll
    for (int a = 0; a < MB256; ++a)
#pragma unroll
        for (int b = 0; b < MB256; ++b) mma2<PREC>(acc[a][b], fa[a], fb[b]);
}

// One K slice, software-pipelined across slices. On entry f0a/f0b hold k-group
// 0 of this slice (stage `cur`). The step
//   1. multiplies k-group 0 while it reads k-group 1 from `cur` and issues the
//      loads of the slice three ahead into `wr` (the stage freed last step);
//   2. waits until the next stage has landed and every wave is done reading
//      `cur`, and synchronises;
//   3. multiplies k-group 1 while it reads k-group 0 of the next stage `nxt`
//      into f0a/f0b for the following step. (The tile loop reads k-group 0
//      of a tile again at its start, so the read-ahead of a tile's last step
//      is dead once the tile ends and the fragments are not held in
//      registers through the epilogue.)
// The three stages arrive as restrict pointers: once inlined their accesses
// carry distinct alias scopes, so LDS reads never wait for the loads in flight.
// LANDED: k-group 1 of `cur` is read by read_group_landed (the first step of a
// tile that starts at stage 2).
template <int PREC, bool LANDED = false>
__device__ __forceinline__ void slice_step(typename A2<PREC>::T (&acc)[MB256][MB256], Frags<PREC> &f0a,
                                           Frags<PREC> &f0b, const TileAddr &ia, int is, int wave, int wm, int wn,
                                           int lrow, int lhalf, const unsigned char *__restrict__ cur,
                                           const unsigned char *__restrict__ nxt, unsigned char *__restrict__ wr)
{
    constexpr int MPG = (PREC == P_F32 ? 4 : 1) * MB256 * MB256;  // MFMAs per k-group
    Frags<PREC> f1a, f1b;
    issue_slice(ia, is, wave, wr);
    if constexpr (LANDED) read_group_landed<PREC>(f1a, f1b, cur, 1, wm, wn, lrow, lhalf);
    else read_group<PREC>(f1a, f1b, cur, 1, wm, wn, lrow, lhalf);
    mma_group<PREC>(acc, f0a, f0b);
#pragma unroll
    for (int k = 0; k < 2 * MB256; ++k) {
        __builtin_amdgcn_sched_group_barrier(SG_MFMA, MPG / (2 * MB256), 0);
        __builtin_amdgcn_sched_group_barrier(SG_DS_READ, 1, 0);
        __builtin_amdgcn_sched_group_barrier(SG_VMEM_READ, 1, 0);
    }
    __builtin_amdgcn_s_waitcnt(WAIT_SLICE);
    __builtin_amdgcn_s_barrier();
    read_group<PREC>(f0a, f0b, nxt, 0, wm, wn, lrow, lhalf);
    mma_group<PREC>(acc, f1a, f1b);
#pragma unroll
    for (int k = 0; k < 2 * MB256; ++k) {
        __builtin_amdgcn_sched_group_barrier(SG_DS_READ, 1, 0);
        __builtin_amdgcn_sched_group_barrier(SG_MFMA, MPG / (2 * MB256), 0);
    }
}

// Folded row scalars (BF16 and FP32 screens): operands of one extra
// matrix-core step per accumulator block whose product is -(s^_i + s^_j)/2,
// so that the accumulator ends at fl(-(s^_i + s^_j)/2 + <x~_i, x~_j>) and
// D~ = -2 acc (bound.h, folded form).
//   BF16 (K = 16 per step; lane half h holds k = 8h .. 8h+7): with c = -s^/4
//   split into three BF16 parts (c1, c2, c3), the A row of a lane in half 0
//   holds [c1 c2 c3 1 1 1 0 0] and in half 1 [1 1 1 c1 c2 c3 0 0]; the B row
//   the other pattern. Both halves then contribute c_i + c_j.
//   FP32 (K = 2; lane half h holds k = h): A = (c_i, 1), B = (1, c_j) with
//   c = -s^/2.
// BF16 fragment [c1 c2 c3 1 1 1 0 0] (first) or [1 1 1 c1 c2 c3 0 0] from the
// row's folded scalar words w0 = c1 | c2 << 16, w1 = c3 | 1.0 << 16 (written
// by the builder, fold_words).
__device__ __forceinline__ u32x4 fold_frag_words(uint32_t w0, uint32_t w1, bool first)
{
    constexpr uint32_t ONE2 = 0x3f803f80u;
    const uint32_t q1 = 0x3f80u | (w0 << 16);
    const uint32_t q2 = __builtin_amdgcn_alignbit(w1, w0, 16);
    // per-dword selects (the lane half is divergent: no branches); the zero
    // dword is materialised here rather than shared with a loop-wide zero
    // register (which the allocator would spill with it)
    uint32_t z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    return u32x4{first ? w0 : ONE2, first ? w1 : q1, first ? ONE2 : q2, z};
}

// MASKED = false: every pair of every listed tile is admissible (the host
// lists such full tiles apart), so the epilogue carries no masking code.
// K2 = false: every listed problem's rows hold a multiple of four K slices, so
// every tile starts at stage 0 of the ring. K2 = true: a multiple of two (rows
// of 128 bytes, e.g. BF16 windows of 64 values, are not padded to 256), so a
// tile starts at stage 0 or 2 and the slice loop turns two slices at a time.
template <int PREC, int MODE, bool MASKED, bool K2>
__global__ __launch_bounds__(256, 1) __attribute__((amdgpu_waves_per_eu(1, 1))) void screen256_kernel(ScreenArgs args)
{
    using AccT = typename A2<PREC>::T;
    using S = typename A2<PREC>::S;
    constexpr S SINF = PREC == P_I8 ? (S)0x7fffffff : (S)INFINITY;
    constexpr int ESZ = PREC == P_F32 ? 4 : (PREC == P_BF16 ? 2 : 1);
    constexpr bool FOLD = PREC != P_I8;  // row scalars folded into the product

    // row scalars of blocks I and J, double-buffered by tile parity: the
    // scalars of the next tile are loaded while the current one is screened.
    // BF16: the two folded-scalar words of each row; else s^ (one word)
    constexpr int SW = PREC == P_BF16 ? 2 : 1;
    __shared__ __attribute__((aligned(16))) uint32_t sh_w[2 * 2 * T256 * SW];
    S *const sh_s = (S *)sh_w;
    // source positions of the rows of blocks I and J (windows of a series in
    // reference order; same double buffering), for the exclusion zone
    __shared__ __attribute__((aligned(16))) int32_t sh_o[2 * 2 * T256];

    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int wm = wave >> 1, wn = wave & 1;

    // 32-bit tile indices (the host keeps lists below 2^31 entries), so that
    // the loop bookkeeping stays in scalar registers and scalar compares
    const bool dense = (MODE & M_EMIT) && args.sel_dense && (int64_t)*args.sel_count * 4 > args.ntiles;
    const int32_t count =
        (MODE & M_EMIT) && !dense ? (int32_t)*args.sel_count : (int32_t)args.ntiles;
    const int32_t stride = (int32_t)gridDim.x;

    c_u64 *tiles = (c_u64 *)(dense ? args.sel_dense : args.tiles);
    auto next_valid = [&](int32_t t) -> int32_t {
        while (t < count && tiles[t] == TILE_NONE) t += stride;
        return t;
    };
    // direct-to-LDS load of the row scalars of tile `tt` (blocks I and J) into
    // sh_s half `half`: each wave loads 64 of block I and 64 of block J
    auto load_scalars = [&](int32_t tt, int half) {
        const uint64_t e = tiles[tt];
        const c_prob &Q = ((c_prob *)args.probs)[tile_prob(e)];
        const uint32_t lo = (uint32_t)fresh_lane() * 4;
        if constexpr (PREC == P_BF16) {
            // 64 rows x 8 bytes of block I and of block J: two 256-byte loads each
            const unsigned char *fb = (const unsigned char *)Q.fold;
            uint32_t *dst = sh_w + half * (2 * T256 * 2);
            // (the second 256 bytes of each by the instruction offset, which
            // moves the global and the LDS address alike)
            const unsigned char *gi = fb + ((int64_t)tile_I(e) * T256 + wave * 64) * 8 + lo;
            const unsigned char *gj = fb + ((int64_t)tile_J(e) * T256 + wave * 64) * 8 + lo;
            __builtin_amdgcn_global_load_lds((g_void *)gi, (lds_void *)(dst + wave * 128), 4, 0, 0);
            __builtin_amdgcn_global_load_lds((g_void *)gi, (lds_void *)(dst + wave * 128), 4, 256, 0);
            __builtin_amdgcn_global_load_lds((g_void *)gj, (lds_void *)(dst + 2 * T256 + wave * 128), 4, 0, 0);
            __builtin_amdgcn_global_load_lds((g_void *)gj, (lds_void *)(dst + 2 * T256 + wave * 128), 4, 256, 0);
        } else {
            const unsigned char *sb = (const unsigned char *)Q.shat;
            S *dst = sh_s + half * (2 * T256);
            __builtin_amdgcn_global_load_lds((g_void *)(sb + ((int64_t)tile_I(e) * T256 + wave * 64) * 4 + lo),
                                             (lds_void *)(dst + wave * 64), 4, 0, 0);
            __builtin_amdgcn_global_load_lds((g_void *)(sb + ((int64_t)tile_J(e) * T256 + wave * 64) * 4 + lo),
                                             (lds_void *)(dst + T256 + wave * 64), 4, 0, 0);
        }
        if constexpr (MASKED) {
            if (Q.perm && Q.motif) {
                // the permutation is padded to whole blocks by the host; the
                // lane's byte offset is rebuilt here as a 64-bit value (a
                // widened one kept from elsewhere would be held, and spilled,
                // across the tile loop)
                const unsigned char *pb = (const unsigned char *)Q.perm;
                int32_t *od = sh_o + half * (2 * T256);
                const uint64_t lo64 = fresh_lane_bytes4();
                __builtin_amdgcn_global_load_lds((g_void *)(pb + ((int64_t)tile_I(e) * T256 + wave * 64) * 4 + lo64),
                                                 (lds_void *)(od + wave * 64), 4, 0, 0);
                __builtin_amdgcn_global_load_lds((g_void *)(pb + ((int64_t)tile_J(e) * T256 + wave * 64) * 4 + lo64),
                                                 (lds_void *)(od + T256 + wave * 64), 4, 0, 0);
            }
        }
    };

    // Pass 2's radius candidates: each wave takes output slots in slabs of
    // SLAB (one atomic add per slab, not one per emission: at volume the
    // candidates number millions and the counter is one word); the unused
    // end of a slab is marked empty (problem index ~0) for the verifier.
    constexpr uint32_t SLAB = 256;
    uint64_t slab = 0;        // first slot of the wave's slab (wave-uniform)
    uint32_t slab_used = SLAB;
    uint32_t nIn = 0;         // pairs proved inside the radius by their screen value (counting form)
    auto close_slab = [&]() {
        // entries [slab_used, SLAB) of the current slab: empty
        const uint32_t l = (uint32_t)fresh_lane();
        for (uint32_t k = slab_used + l; k < SLAB; k += 64)
            if (slab + k < args.capR) args.candR[slab + k] = Cand{0, 0, 0.0f, 0xffffffffu};
    };
    auto emit_r = [&](bool pred, const Cand &cd) {
        const uint64_t m = __ballot(pred);
        if (m == 0) return;
        const uint32_t n = (uint32_t)__popcll(m);
        if (slab_used + n > SLAB) {
            if (slab_used < SLAB) close_slab();
            u64c base = 0;
            if (fresh_lane() == 0) base = atomicAdd(args.cntR, (u64c)SLAB);
            slab = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
            slab_used = 0;
        }
        const uint32_t rank =
            __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (pred && slab + slab_used + rank < args.capR) args.candR[slab + slab_used + rank] = cd;
        slab_used += n;
    };

    int32_t t = next_valid((int32_t)blockIdx.x);
    if (t >= count) return;
    int tcount = 0;
    load_scalars(t, 0);

    // load cursor: runs three slices ahead of the multiply, across tiles; at
    // the end of the list it keeps re-reading its last slice (always in bounds)
    int32_t it = t;
    int is = 0;
    TileAddr ia = tile_addr<ESZ>(args, tiles[it]);
    auto advance = [&]() {
        if (is + 1 < ia.nst) {
            ++is;
        } else {
            const int32_t tn = next_valid(it + stride);
            if (tn < count) {
                it = tn;
                is = 0;
                ia = tile_addr<ESZ>(args, tiles[it]);
            }
        }
    };
    issue_slice(ia, is, wave, stage_ptr<0>());
    advance();
    issue_slice(ia, is, wave, stage_ptr<1>());
    advance();
    issue_slice(ia, is, wave, stage_ptr<2>());
    advance();
    // the first tile's scalars are older than the last 16 loads: landed
    __builtin_amdgcn_s_waitcnt(WAIT_SLICE);
    __builtin_amdgcn_s_barrier();
    [[maybe_unused]] int ph = 0;   // K2: ring stage (0 or 2) of the current tile's first slice
    // The tile loop; the tile body is included once per ring stage a tile may
    // start at (one for K2 = false).
    while (t < count) {
        if (!K2 || ph == 0) {
#define CPMI_TILE_P0 0
#include "screen256_tile.inc"
#undef CPMI_TILE_P0
        } else {
#define CPMI_TILE_P0 2
#include "screen256_tile.inc"
#undef CPMI_TILE_P0
        }
    }
    if constexpr (MODE & M_EMIT) {
        if (slab_used < SLAB) close_slab();
        if (args.cntIn) wave_count(args.cntIn, nIn);
    }
    // the load cursor keeps loads in flight past the last tile: let them land
    // before the work-group (and its LDS) is released
    __builtin_amdgcn_s_waitcnt(0);
}

template <int PREC, bool K2>
static void launch256k(int mode, bool masked, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    dim3 g((unsigned)grid), b(256);
    if (mode == M_MIN && !masked) hipLaunchKernelGGL((screen256_kernel<PREC, M_MIN, false, K2>), g, b, 0, st, a);
    else if (mode == M_MIN) hipLaunchKernelGGL((screen256_kernel<PREC, M_MIN, true, K2>), g, b, 0, st, a);
    else if (mode == M_DUMP) hipLaunchKernelGGL((screen256_kernel<PREC, M_DUMP, true, K2>), g, b, 0, st, a);
    else hipLaunchKernelGGL((screen256_kernel<PREC, M_EMIT, true, K2>), g, b, 0, st, a);
}

template <int PREC>
static void launch256(int mode, bool masked, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    if (a.k2) launch256k<PREC, true>(mode, masked, a, grid, st);
    else launch256k<PREC, false>(mode, masked, a, grid, st);
}

void launch_screen256(int prec, int mode, bool masked, const ScreenArgs &a, int64_t grid, hipStream_t st)
{
    if (grid <= 0) return;
    if (prec == P_F32) launch256<P_F32>(mode, masked, a, grid, st);
    else if (prec == P_BF16) launch256<P_BF16>(mode, masked, a, grid, st);
    else launch256<P_I8>(mode, masked, a, grid, st);
}

}  // namespace cpmi
