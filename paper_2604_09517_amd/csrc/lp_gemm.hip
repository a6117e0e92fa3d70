// Trailing update of the low-precision LU on the matrix cores (gfx950).
//
// Sec. III-A.2: the trailing matrix updates run in reduced precision; the
// paper's runs store the matrix in BF16 and accumulate products in FP32.
//   16-bit form:  A22 <- round( fp32(A22) - L21 U12 ), bf16 or fp16 operands,
//                 v_mfma_f32_16x16x32_{bf16,f16}, accumulators start at A22.
//   FP8 form:     A22 <- round_fp16( fp32(A22) - (Lq Uq) sL sU ), e4m3fn
//                 operands with one power-of-two scale per tile of rows of L21
//                 and of columns of U12, v_mfma_scale_f32_16x16x128_f8f6f4
//                 with unit block scales.
//
// Operands come chunk-packed (one K chunk of one tile is one contiguous
// block) and are staged through LDS rings filled by direct global->LDS
// loads; see each form below for its tile and ring.
//
// MFMA lane layouts (measured on gfx950; lane l, i = l % 16, g = l / 16):
//   16x16x32 16-bit: A lane holds A[i][8g .. 8g+7], B lane B[8g .. 8g+7][i],
//   16x16x128 fp8:   A lane holds A[i][16g .. 16g+15] in bytes 0-15 and
//                    A[i][64+16g .. 64+16g+15] in bytes 16-31, B likewise;
//                    the block-scaled form takes the scale byte of lane
//                    (i, g) for row i of A (column i of B) and the k block
//                    32g .. 32g+31,
//   both: accumulator register r holds D[4g + r][i].
#include <hip/hip_runtime.h>

#include "common.h"
#include "lp_common.h"
#include "lp_kernels.h"

namespace {

using namespace mxlu;

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

constexpr int TM = 256, TN = 128;

// Tile of workgroup g: consecutive workgroup ids go to the eight XCDs in
// turn, so each XCD takes a contiguous range of the tile order, in which
// groups of GM tile rows are walked column by column (the operand panels of
// the tiles an XCD runs at once stay in its L2).
template <int GM>
__device__ inline void tile_of(int g, int tiles_m, int tiles_n, int &tm, int &tn) {
    const int G = tiles_m * tiles_n;
    const int per = G / 8, rem = G % 8;
    const int xcd = g % 8, local = g / 8;
    const int t = (xcd < rem) ? xcd * (per + 1) + local
                              : rem * (per + 1) + (xcd - rem) * per + local;
    const int in_group = GM * tiles_n;
    const int group = t / in_group;
    const int first_m = group * GM;
    const int gsize = min(tiles_m - first_m, GM);
    const int r = t - group * in_group;
    tm = first_m + r % gsize;
    tn = r / gsize;
}

template <int FMT>
__device__ __forceinline__ v4f mfma16(uint4 a, uint4 b, v4f c) {
    if constexpr (FMT == kFmtBf16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                       __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(v8h, a),
                                                      __builtin_bit_cast(v8h, b), c, 0, 0, 0);
}

// ------------------------------------------------------------ 16-bit form
// Operands come chunk-packed (one K chunk of 32 of a tile = one contiguous
// block: 16 KB of L21, 8 KB of U12) and are copied to an LDS ring of kNs16
// stages with 16-byte direct global->LDS loads (no register staging): each
// wave issues 4 + 2 loads of 1 KB per chunk, so up to kNs16 - 1 chunks are in
// flight while the matrix cores work on the current one, and one workgroup
// barrier per chunk orders the ring.  A is negated when read from LDS.  The
// A rows of each pair of MFMA blocks are interleaved so that a lane's
// accumulators cover 8 consecutive rows of a column: C is read and written
// 16 bytes per lane.
constexpr int BK16 = kLpKc;
constexpr int kNs16 = 3;
static_assert(TM == kLpTileM && TN == kLpTileN, "tile and packing must agree");

typedef __attribute__((address_space(1))) void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;
typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

// 16 bytes of the C tile, optionally as streaming (non-temporal) accesses:
// each C element is touched once per update, and keeping it out of the caches
// leaves them to the operand panels that every tile of a tile row or column
// reads again.  Measured: the FP8 update gains with both (11.1 -> 9.5-9.9 ms
// per launch at N = 131072, NB = 1024; loads or stores alone are slower than
// neither), the 16-bit update loses with any (2.29 -> 2.34-2.43 ms at
// N = 65536, NB = 512), so it keeps ordinary accesses.
template <bool NT>
__device__ __forceinline__ uint4 c_load(const uint16_t *p) {
    if constexpr (!NT) return *reinterpret_cast<const uint4 *>(p);
    const v4u v = __builtin_nontemporal_load(reinterpret_cast<const v4u *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
template <bool NT>
__device__ __forceinline__ void c_store(uint16_t *p, uint4 v) {
    if constexpr (!NT) {
        *reinterpret_cast<uint4 *>(p) = v;
        return;
    }
    __builtin_nontemporal_store(v4u{v.x, v.y, v.z, v.w}, reinterpret_cast<v4u *>(p));
}

// LDS byte address of a pointer into a __shared__ array
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)reinterpret_cast<uintptr_t>((const lvoid_t *)p);
}

// Operand fragments of one K chunk read from the LDS ring.  These reads are
// written as one assembly block that waits for its own results (lgkmcnt(0))
// because the compiler cannot tell the ring stage read here from the stages
// that the direct global->LDS copies of later chunks are still filling: it
// would put a wait for every outstanding copy (vmcnt(0)) before the first
// read, which leaves no copy in flight while the matrix cores run.  The
// ring's own vmcnt wait and workgroup barrier order these reads after the
// copies of the chunk they read.  The outputs are early-clobber: a read is
// issued before the later reads have taken their addresses.
//
// 16-bit form: a[i] at a0 + 1024 i (i < 8), b[j] at b0 + 1024 j (j < 4).
__device__ __forceinline__ void lds_frags16(uint32_t a0, uint32_t b0, uint4 (&a)[8],
                                            uint4 (&b)[4]) {
    v4i x[12];
    asm volatile(
        "ds_read_b128 %0, %12\n\t"
        "ds_read_b128 %1, %12 offset:1024\n\t"
        "ds_read_b128 %2, %12 offset:2048\n\t"
        "ds_read_b128 %3, %12 offset:3072\n\t"
        "ds_read_b128 %4, %12 offset:4096\n\t"
        "ds_read_b128 %5, %12 offset:5120\n\t"
        "ds_read_b128 %6, %12 offset:6144\n\t"
        "ds_read_b128 %7, %12 offset:7168\n\t"
        "ds_read_b128 %8, %13\n\t"
        "ds_read_b128 %9, %13 offset:1024\n\t"
        "ds_read_b128 %10, %13 offset:2048\n\t"
        "ds_read_b128 %11, %13 offset:3072\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]),
          "=&v"(x[7]), "=&v"(x[8]), "=&v"(x[9]), "=&v"(x[10]), "=&v"(x[11])
        : "v"(a0), "v"(b0));
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = __builtin_bit_cast(uint4, x[i]);
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = __builtin_bit_cast(uint4, x[8 + j]);
}

// FP8 form: fragment i (i < 4) of A is 16 bytes at alo + 2048 i and 16 at
// ahi + 2048 i, likewise B from blo / bhi.
__device__ __forceinline__ void lds_frags8(uint32_t alo, uint32_t ahi, uint32_t blo, uint32_t bhi,
                                           v8i (&a)[4], v8i (&b)[4]) {
    v4i x[16];
    asm volatile(
        "ds_read_b128 %0, %16\n\t"
        "ds_read_b128 %1, %17\n\t"
        "ds_read_b128 %2, %16 offset:2048\n\t"
        "ds_read_b128 %3, %17 offset:2048\n\t"
        "ds_read_b128 %4, %16 offset:4096\n\t"
        "ds_read_b128 %5, %17 offset:4096\n\t"
        "ds_read_b128 %6, %16 offset:6144\n\t"
        "ds_read_b128 %7, %17 offset:6144\n\t"
        "ds_read_b128 %8, %18\n\t"
        "ds_read_b128 %9, %19\n\t"
        "ds_read_b128 %10, %18 offset:2048\n\t"
        "ds_read_b128 %11, %19 offset:2048\n\t"
        "ds_read_b128 %12, %18 offset:4096\n\t"
        "ds_read_b128 %13, %19 offset:4096\n\t"
        "ds_read_b128 %14, %18 offset:6144\n\t"
        "ds_read_b128 %15, %19 offset:6144\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(x[0]), "=&v"(x[1]), "=&v"(x[2]), "=&v"(x[3]), "=&v"(x[4]), "=&v"(x[5]), "=&v"(x[6]),
          "=&v"(x[7]), "=&v"(x[8]), "=&v"(x[9]), "=&v"(x[10]), "=&v"(x[11]), "=&v"(x[12]),
          "=&v"(x[13]), "=&v"(x[14]), "=&v"(x[15])
        : "v"(alo), "v"(ahi), "v"(blo), "v"(bhi));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        a[i] = v8i{x[2 * i].x, x[2 * i].y, x[2 * i].z, x[2 * i].w,
                   x[2 * i + 1].x, x[2 * i + 1].y, x[2 * i + 1].z, x[2 * i + 1].w};
        b[i] = v8i{x[8 + 2 * i].x, x[8 + 2 * i].y, x[8 + 2 * i].z, x[8 + 2 * i].w,
                   x[9 + 2 * i].x, x[9 + 2 * i].y, x[9 + 2 * i].z, x[9 + 2 * i].w};
    }
}

__device__ __forceinline__ uint4 neg16(uint4 v) {   // flip the sign bit of 8 16-bit values
    v.x ^= 0x80008000u;
    v.y ^= 0x80008000u;
    v.z ^= 0x80008000u;
    v.w ^= 0x80008000u;
    return v;
}

template <int FMT, bool NTL = false, bool NTS = false>
__global__ __launch_bounds__(256, 2) void lp_schur16_kernel(
    int64_t M, int64_t N, int K, const uint16_t *__restrict__ Lp, int64_t Mp,
    const uint16_t *__restrict__ Up, int64_t Np, uint16_t *__restrict__ C, int64_t ldc,
    int tiles_m, int tiles_n) {
    constexpr int SA = TM * BK16, SB = TN * BK16;   // elements per stage
    __shared__ __attribute__((aligned(1024))) uint16_t ring[kNs16][SA + SB];

    int tm, tn;
    tile_of<8>(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * TM, col0 = (int64_t)tn * TN;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lg = lane >> 4;

    // Row mapping: the A operand of MFMA block bi = 2p + h supplies, in lane
    // li, tile row 32p + 2 li + h, so accumulator register r of lane (li, lg)
    // of blocks 2p and 2p + 1 holds the 8 consecutive rows 32p + 8 lg + 2r + h
    // of column c: C moves 16 bytes per lane (rows row8 .. row8 + 7).
    // Interior tiles with 16-byte aligned columns (uniform branch) issue all
    // their loads back to back without checks.
    const bool full = row0 + TM <= M && col0 + TN <= N && (ldc & 7) == 0 &&
                      ((uintptr_t)C & 15) == 0;
    auto row_of = [&](int bi, int r) -> int64_t {
        return row0 + wm * 128 + 32 * (bi >> 1) + 2 * (4 * lg + r) + (bi & 1);
    };
    v4f acc[8][4];
    if (full) {
#pragma unroll
        for (int pr = 0; pr < 4; ++pr)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t r8 = row0 + wm * 128 + 32 * pr + 8 * lg;
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
                const uint4 v = c_load<NTL>(&C[(size_t)r8 + (size_t)c * ldc]);
                const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    acc[2 * pr][bj][r] = lp_to_f32<FMT>((uint16_t)w4[r]);
                    acc[2 * pr + 1][bj][r] = lp_to_f32<FMT>((uint16_t)(w4[r] >> 16));
                }
            }
    } else {
#pragma unroll
        for (int bi = 0; bi < 8; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row_of(bi, r);
                    acc[bi][bj][r] = (row < M && c < N)
                                         ? lp_to_f32<FMT>(C[(size_t)row + (size_t)c * ldc])
                                         : 0.0f;
                }
            }
    }

    // LDS layout of a stage: 64-byte lines (one row of L21 or column of U12
    // over the chunk's 32 k), four 16-byte segments.  The 16 lanes li of a
    // lane group read one segment of 16 lines at once (one pass of a 16-byte
    // LDS read), so (1) the A rows 32p + 2 li + h of one MFMA block sit in the
    // consecutive lines 32p + 16h + li, and (2) segment s of line x is stored
    // in slot s ^ sw(x), sw(x) = ((x >> 1) & 3) ^ ((x >> 3) & 1): the 16 lanes
    // of a pass touch 16 distinct 16-byte bank groups of 256 bytes (8 in each
    // half).  Wave w copies lines [64 w, 64 w + 64) of L21 and [32 w, 32 w +
    // 32) of U12, slots in lane order; each lane fetches the global segment
    // that belongs in its slot (4 lanes per contiguous 64-byte global line).
    auto sw = [](int x) { return ((x >> 1) & 3) ^ ((x >> 3) & 1); };
    const int t4 = lane >> 2, s4 = lane & 3;
    int offA[4], offB[2];   // byte offsets of this lane's global segments in a chunk
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = wave * 64 + 16 * q + t4;
        const int r = 32 * (x >> 5) + 2 * (x & 15) + ((x >> 4) & 1);
        offA[q] = r * (BK16 * 2) + 16 * (s4 ^ sw(x));
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int x = wave * 32 + 16 * q + t4;
        offB[q] = x * (BK16 * 2) + 16 * (s4 ^ sw(x));
    }
    const char *gA = reinterpret_cast<const char *>(Lp + (size_t)row0 * BK16);
    const char *gB = reinterpret_cast<const char *>(Up + (size_t)col0 * BK16);
    const size_t strideA = (size_t)Mp * BK16 * sizeof(uint16_t);   // bytes per K chunk
    const size_t strideB = (size_t)Np * BK16 * sizeof(uint16_t);
    auto issue = [&](int kc, int st) {
        const char *ga = gA + (size_t)kc * strideA;
        const char *gb = gB + (size_t)kc * strideB;
        char *la = reinterpret_cast<char *>(&ring[st][0]) + wave * 4096;
        char *lb = reinterpret_cast<char *>(&ring[st][SA]) + wave * 2048;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            __builtin_amdgcn_global_load_lds((gvoid_t *)(ga + offA[q]), (lvoid_t *)(la + q * 1024),
                                             16, 0, 0);
#pragma unroll
        for (int q = 0; q < 2; ++q)
            __builtin_amdgcn_global_load_lds((gvoid_t *)(gb + offB[q]), (lvoid_t *)(lb + q * 1024),
                                             16, 0, 0);
    };

    const int nk = K / BK16;
#pragma unroll
    for (int c = 0; c < kNs16 - 1; ++c)
        if (c < nk) issue(c, c);
    for (int kt = 0; kt < nk; ++kt) {
        // chunk kt has landed once at most min(kNs16 - 2, nk - 1 - kt) later
        // chunks (6 loads each) are outstanding; the C loads came first
        static_assert(kNs16 == 3, "the wait below assumes three stages");
        if (kt + 1 < nk) __builtin_amdgcn_s_waitcnt(0x0F70 | 6);   // vmcnt(6)
        else __builtin_amdgcn_s_waitcnt(0x0F70);                   // vmcnt(0)
        __syncthreads();   // every wave's part of chunk kt; stage (kt - 1) % 3 free
        if (kt + kNs16 - 1 < nk) issue(kt + kNs16 - 1, (kt + kNs16 - 1) % kNs16);
        const uint16_t *as = &ring[kt % kNs16][0];
        const uint16_t *bs = &ring[kt % kNs16][SA];
        // lines read are 16-aligned plus li, so their swizzle is sw(li)
        const int so = 8 * (lg ^ sw(li));
        // A block bi at line wm 128 + 16 bi + li, B block bj at wn 64 + 16 bj + li
        uint4 a[8], b[4];
        lds_frags16(lds_addr(&as[(wm * 128 + li) * BK16 + so]),
                    lds_addr(&bs[(wn * 64 + li) * BK16 + so]), a, b);
#pragma unroll
        for (int bi = 0; bi < 8; ++bi) a[bi] = neg16(a[bi]);
#pragma unroll
        for (int bi = 0; bi < 8; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma16<FMT>(a[bi], b[bj], acc[bi][bj]);
    }

    if (full) {
#pragma unroll
        for (int pr = 0; pr < 4; ++pr)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t r8 = row0 + wm * 128 + 32 * pr + 8 * lg;
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
                uint32_t w4[4];
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    w4[r] = (uint32_t)f32_to_lp<FMT>(acc[2 * pr][bj][r]) |
                            ((uint32_t)f32_to_lp<FMT>(acc[2 * pr + 1][bj][r]) << 16);
                c_store<NTS>(&C[(size_t)r8 + (size_t)c * ldc], make_uint4(w4[0], w4[1], w4[2], w4[3]));
            }
    } else {
#pragma unroll
        for (int bi = 0; bi < 8; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row_of(bi, r);
                    if (row < M && c < N)
                        C[(size_t)row + (size_t)c * ldc] = f32_to_lp<FMT>(acc[bi][bj][r]);
                }
            }
    }
}

// ------------------------------------------------------------ FP8 form
// A 4-wave workgroup owns a 128 x 128 tile (each wave 64 x 64 = 4 x 4 MFMA
// blocks); two workgroups per CU.  One K chunk is 128 values (one MFMA K
// step): 16 KB of L21 and 16 KB of U12, copied into a two-stage LDS ring with
// 16-byte direct global->LDS loads (8 loads of 1 KB per wave and chunk).
// The accumulators start at zero and take +Lq Uq; the epilogue forms
// C - acc sL sU (the scalings exact: powers of two), the order of the
// definition; C is read and written 16 bytes (8 rows) per lane, the A rows of
// each pair of MFMA blocks being interleaved as in the 16-bit form.
constexpr int kTm8 = 128, kTn8 = 128;
constexpr int BK8 = kLp8Kc;
static_assert(kTm8 == kLp8Tile && kTn8 == kLp8Tile, "tile and packing must agree");

// vmcnt(n) for the waits of the rings below (gfx9 encoding: vmcnt bits [3:0]
// and [15:14], expcnt and lgkmcnt left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt(0x0F70 | (N & 15) | ((N >> 4) << 14));
}

// MX: instead of the tile scales, one E8M0 scale byte per line and block of
// 32 k (sLx[b Mp + r], sUx[b Np + c]) goes to the matrix cores with the
// operands: lane (li, lg) supplies the byte of block lg of the chunk for its
// row (column), the operand bytes being placed so that the matrix cores' k
// is the chunk's k (bytes 0-15 of a lane from k 16 lg, bytes 16-31 from
// k 64 + 16 lg); the epilogue is then C - acc.
template <int FMT, int NS, bool MX, bool NTL = true, bool NTS = true>
__global__ __launch_bounds__(256, NS <= 2 ? 2 : 1) void lp_schur8_kernel(
    int64_t M, int64_t N, int K, const uint8_t *__restrict__ Lq, int64_t Mp,
    const float *__restrict__ sL, const uint8_t *__restrict__ Uq, int64_t Np,
    const float *__restrict__ sU, int tile, const uint8_t *__restrict__ sLx,
    const uint8_t *__restrict__ sUx, uint16_t *__restrict__ C, int64_t ldc, int tiles_m,
    int tiles_n) {
    static_assert(!MX || NS == 2, "the MX scale loads are waited for with the chunk (vmcnt(0))");
    constexpr int kNs8 = NS;
    constexpr int SA = kTm8 * BK8, SB = kTn8 * BK8;   // bytes per stage
    constexpr int NA = SA / 4 / 1024, NB = SB / 4 / 1024;
    __shared__ __attribute__((aligned(1024))) uint8_t ring[kNs8][SA + SB];

    int tm, tn;
    tile_of<16>(blockIdx.x, tiles_m, tiles_n, tm, tn);
    const int64_t row0 = (int64_t)tm * kTm8, col0 = (int64_t)tn * kTn8;
    // scale-tile index of a row or column (32-bit; a shift for power-of-two tiles)
    const bool pow2 = (tile & (tile - 1)) == 0;
    const int tshift = __builtin_ctz((unsigned)tile);
    auto tix = [&](int64_t x) {
        return pow2 ? (int)((uint32_t)x >> tshift) : (int)((uint32_t)x / (uint32_t)tile);
    };
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 15, lg = lane >> 4;

    // Rows as in the 16-bit form: the A operand of MFMA block bi = 2p + h
    // supplies tile row 32p + 2 li + h in lane li, so a lane's accumulators of
    // blocks 2p, 2p + 1 cover 8 consecutive rows of one column (16 bytes of C;
    // rows 0-3 and 4-7 each share a scale tile, tiles being multiples of 4).
    // The accumulators start at zero and the epilogue forms C - acc sL sU (the
    // scalings are exact: powers of two), so the C tile is needed only at the
    // end: interior tiles with 16-byte aligned columns (uniform branch) load it
    // just before the first operand chunks, and its latency overlaps theirs.
    const bool full = row0 + kTm8 <= M && col0 + kTn8 <= N && (ldc & 7) == 0 &&
                      ((uintptr_t)C & 15) == 0;
    auto row_of = [&](int bi, int r) -> int64_t {
        return row0 + wm * 64 + 32 * (bi >> 1) + 2 * (4 * lg + r) + (bi & 1);
    };
    v4f acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    uint4 cv[2][4];

    // LDS layout of a stage: 128-byte lines (one row of L21 or column of U12
    // over the chunk's 128 k), 16-byte segments.  A row is read by the 16
    // lanes li of a lane group at once (one pass of a 16-byte LDS read), so
    // (1) the A rows 32p + 2 li + h that one MFMA block takes sit in 16
    // consecutive lines, line 32p + 16h + li, and (2) segment s of line x is
    // stored in slot s ^ sw(x), sw(x) = (x & 7) ^ ((x >> 3) & 1): the 16 lanes
    // of a pass then touch 16 distinct 16-byte bank groups of the 256 bytes
    // the LDS serves per cycle (and 8 distinct ones in each half).  The
    // global->LDS copy writes slots in lane order, so each lane fetches the
    // global segment that belongs in its slot; the 8 lanes of a line still
    // read one contiguous 128-byte global line.
    auto sw = [](int x) { return (x & 7) ^ ((x >> 3) & 1); };
    const int t8 = lane >> 3, s8 = lane & 7;
    int offA[NA], offB[NB];   // byte offsets of this lane's global segments in a chunk
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int x = wave * (SA / 4 / BK8) + 8 * q + t8;            // LDS line
        const int r = 32 * (x >> 5) + 2 * (x & 15) + ((x >> 4) & 1);   // tile row
        offA[q] = r * BK8 + 16 * (s8 ^ sw(x));
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int x = wave * (SB / 4 / BK8) + 8 * q + t8;
        offB[q] = x * BK8 + 16 * (s8 ^ sw(x));
    }
    const char *gA = reinterpret_cast<const char *>(Lq + (size_t)row0 * BK8);
    const char *gB = reinterpret_cast<const char *>(Uq + (size_t)col0 * BK8);
    auto issue = [&](int kc, int st) {
        const char *ga = gA + (size_t)kc * Mp * BK8;
        const char *gb = gB + (size_t)kc * Np * BK8;
        char *la = reinterpret_cast<char *>(&ring[st][0]) + wave * (SA / 4);
        char *lb = reinterpret_cast<char *>(&ring[st][SA]) + wave * (SB / 4);
#pragma unroll
        for (int q = 0; q < NA; ++q)
            __builtin_amdgcn_global_load_lds((gvoid_t *)(ga + offA[q]), (lvoid_t *)(la + q * 1024),
                                             16, 0, 0);
#pragma unroll
        for (int q = 0; q < NB; ++q)
            __builtin_amdgcn_global_load_lds((gvoid_t *)(gb + offB[q]), (lvoid_t *)(lb + q * 1024),
                                             16, 0, 0);
    };
    // Line x's 16 bytes at k 16 lg and at k 64 + 16 lg (the matrix cores' k
    // order: segments lg and lg ^ 4); the lines a lane reads are 16-aligned
    // plus li, so sw(x) = sw(li).
    const int so = 16 * (lg ^ sw(li));

    const int nk = K / BK8;
    constexpr int kLoads = NA + NB;   // loads per wave and chunk
    // the C tile's loads go first, so that the ring's waits below count only
    // operand chunks issued after the one they wait for
    if (full) {
#pragma unroll
        for (int pr = 0; pr < 2; ++pr)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t r8 = row0 + wm * 64 + 32 * pr + 8 * lg;
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
                cv[pr][bj] = c_load<NTL>(&C[(size_t)r8 + (size_t)c * ldc]);
            }
    }
#pragma unroll
    for (int c = 0; c < kNs8 - 1; ++c)
        if (c < nk) issue(c, c);
    // MX scale bytes of chunk kc for this lane's four A rows and four B
    // columns (rows beyond M read stale bytes: their outputs are not stored)
    int sa[4] = {127, 127, 127, 127}, sb[4] = {127, 127, 127, 127};
    int sa_n[4], sb_n[4];
    auto load_scales = [&](int kc, int (&a4)[4], int (&b4)[4]) {
        const size_t blk = (size_t)(4 * kc + lg);
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
            a4[bi] = sLx[blk * Mp + (size_t)(row0 + wm * 64 + 32 * (bi >> 1) + 2 * li + (bi & 1))];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
            b4[bj] = sUx[blk * Np + (size_t)(col0 + wn * 64 + bj * 16 + li)];
    };
    if constexpr (MX) load_scales(0, sa, sb);
    for (int kt = 0; kt < nk; ++kt) {
        // chunk kt has landed once at most min(NS - 2, nk - 1 - kt) later
        // chunks are outstanding
        const int later = min(kNs8 - 2, nk - 1 - kt);
        if (kNs8 >= 4 && later >= 2) wait_vmcnt<2 * kLoads>();
        else if (kNs8 >= 3 && later >= 1) wait_vmcnt<kLoads>();
        else wait_vmcnt<0>();
        __syncthreads();   // every wave's part of chunk kt; stage (kt - 1) % NS free
        if (kt + kNs8 - 1 < nk) issue(kt + kNs8 - 1, (kt + kNs8 - 1) % kNs8);
        if constexpr (MX)
            if (kt + 1 < nk) load_scales(kt + 1, sa_n, sb_n);
        const uint8_t *as = &ring[kt % kNs8][0];
        const uint8_t *bs = &ring[kt % kNs8][SA];
        // A block bi at line wm 64 + 16 bi + li, B block bj at wn 64 + 16 bj + li
        v8i a[4], b[4];
        const uint8_t *la = &as[(wm * 64 + li) * BK8], *lb = &bs[(wn * 64 + li) * BK8];
        lds_frags8(lds_addr(la + so), lds_addr(la + (so ^ 64)), lds_addr(lb + so),
                   lds_addr(lb + (so ^ 64)), a, b);
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                    a[bi], b[bj], acc[bi][bj], 0, 0, 0, sa[bi], 0, sb[bj]);
        if constexpr (MX)
            if (kt + 1 < nk)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sa[q] = sa_n[q];
                    sb[q] = sb_n[q];
                }
    }

    // C <- round(fp32(C) - acc sL sU)   (MX: C - acc)
    if (full) {
#pragma unroll
        for (int pr = 0; pr < 2; ++pr)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t r8 = row0 + wm * 64 + 32 * pr + 8 * lg;
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
                float sc_lo = 1.0f, sc_hi = 1.0f;
                if constexpr (!MX) {
                    const float su = sU[tix(c)];
                    sc_lo = sL[tix(r8)] * su;
                    sc_hi = sL[tix(r8 + 4)] * su;
                }
                const uint32_t c4[4] = {cv[pr][bj].x, cv[pr][bj].y, cv[pr][bj].z, cv[pr][bj].w};
                uint32_t w4[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const float sc = r < 2 ? sc_lo : sc_hi;
                    const float lo = lp_to_f32<FMT>((uint16_t)c4[r]) - acc[2 * pr][bj][r] * sc;
                    const float hi =
                        lp_to_f32<FMT>((uint16_t)(c4[r] >> 16)) - acc[2 * pr + 1][bj][r] * sc;
                    w4[r] = (uint32_t)f32_to_lp<FMT>(lo) | ((uint32_t)f32_to_lp<FMT>(hi) << 16);
                }
                c_store<NTS>(&C[(size_t)r8 + (size_t)c * ldc], make_uint4(w4[0], w4[1], w4[2], w4[3]));
            }
    } else {
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) {
                const int64_t c = col0 + wn * 64 + bj * 16 + li;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row_of(bi, r);
                    if (row < M && c < N) {
                        uint16_t *cp = &C[(size_t)row + (size_t)c * ldc];
                        const float sc = MX ? 1.0f : sL[tix(row)] * sU[tix(c)];
                        *cp = f32_to_lp<FMT>(lp_to_f32<FMT>(*cp) - acc[bi][bj][r] * sc);
                    }
                }
            }
    }
}

}  // namespace

namespace mxlu {

int lp_schur_update(int fmt, int64_t M, int64_t N, int K, const uint16_t *Lp, int64_t Mp,
                    int64_t i0, const uint16_t *Up, int64_t Np, int64_t j0, uint16_t *C,
                    int64_t ldc, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    if (K % BK16 || Mp % TM || Np % TN || i0 < 0 || i0 % TM || Mp - i0 < M || j0 < 0 ||
        j0 % TN || Np - j0 < N || ldc % 4 || ((uintptr_t)Lp | (uintptr_t)Up) % 16 ||
        (uintptr_t)C % 8) {
        set_error_msg("lp_schur_update: K % 32, padded packed operands, i0 % 256, j0 % 128, "
                      "ldc % 4 and alignment required");
        return MXLU_E_NOMEM;
    }
    Lp += (size_t)i0 * BK16;   // line i0 of every K chunk
    Up += (size_t)j0 * BK16;
    const int64_t tiles_m = (M + TM - 1) / TM, tiles_n = (N + TN - 1) / TN;
    const dim3 grid((unsigned)(tiles_m * tiles_n));
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL(lp_schur16_kernel<kFmtBf16>, grid, dim3(256), 0, s, M, N, K, Lp, Mp,
                           Up, Np, C, ldc, (int)tiles_m, (int)tiles_n);
    else
        hipLaunchKernelGGL(lp_schur16_kernel<kFmtFp16>, grid, dim3(256), 0, s, M, N, K, Lp, Mp,
                           Up, Np, C, ldc, (int)tiles_m, (int)tiles_n);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_schur_update_fp8(int fmt, int64_t M, int64_t N, int K, const uint8_t *Lq, int64_t Mp,
                        const float *sL, int64_t i0, const uint8_t *Uq, int64_t Np,
                        const float *sU, int64_t j0, int tile, uint16_t *C, int64_t ldc,
                        hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    if (K % BK8 || Mp % kTm8 || Np % kTn8 || tile % 4 || tile <= 0 || i0 < 0 || i0 % kTm8 ||
        i0 % tile || Mp - i0 < M || j0 < 0 || j0 % kTn8 || j0 % tile || Np - j0 < N ||
        ldc % 4 || ((uintptr_t)Lq | (uintptr_t)Uq) % 16 || (uintptr_t)C % 8) {
        set_error_msg("lp_schur_update_fp8: K % 128, padded packed operands, tile % 4, i0 and "
                      "j0 multiples of 128 and of the tile, ldc % 4 and alignment required");
        return MXLU_E_NOMEM;
    }
    Lq += (size_t)i0 * BK8;   // line i0 (j0) of every K chunk
    Uq += (size_t)j0 * BK8;
    sL += i0 / tile;
    sU += j0 / tile;
    const int64_t tiles_m = (M + kTm8 - 1) / kTm8, tiles_n = (N + kTn8 - 1) / kTn8;
    const dim3 grid((unsigned)(tiles_m * tiles_n));
    // two stages with two workgroups per CU: measured faster than three or
    // four stages with one workgroup per CU (11.5 ms against 17.2 and 18.2 ms
    // per launch on average at N = 131072, NB = 1024), whose single wave per
    // SIMD leaves the barrier, the LDS reads and the epilogue exposed, and
    // faster than a 256 x 256 tile with 128 x 128 per wave (11.6 ms); groups
    // of 16 tile rows in the tile order (11.06 ms) against 4, 8 and 32 (11.18,
    // 11.50, 13.00 ms)
    constexpr int kStages = 2;
    const uint8_t *none = nullptr;
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL((lp_schur8_kernel<kFmtBf16, kStages, false>), grid, dim3(256), 0, s, M,
                           N, K, Lq, Mp, sL, Uq, Np, sU, tile, none, none, C, ldc, (int)tiles_m,
                           (int)tiles_n);
    else
        hipLaunchKernelGGL((lp_schur8_kernel<kFmtFp16, kStages, false>), grid, dim3(256), 0, s, M,
                           N, K, Lq, Mp, sL, Uq, Np, sU, tile, none, none, C, ldc, (int)tiles_m,
                           (int)tiles_n);
    MXLU_LAUNCH_CHECK();
    return 0;
}

int lp_schur_update_mx(int fmt, int64_t M, int64_t N, int K, const uint8_t *Lq, int64_t Mp,
                       const uint8_t *sLx, int64_t i0, const uint8_t *Uq, int64_t Np,
                       const uint8_t *sUx, int64_t j0, uint16_t *C, int64_t ldc, hipStream_t s) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
    if (K % BK8 || Mp % kTm8 || Np % kTn8 || i0 < 0 || i0 % kTm8 || Mp - i0 < M || j0 < 0 ||
        j0 % kTn8 || Np - j0 < N || ldc % 4 || ((uintptr_t)Lq | (uintptr_t)Uq) % 16 ||
        (uintptr_t)C % 8 || !sLx || !sUx) {
        set_error_msg("lp_schur_update_mx: K % 128, padded packed operands, scales, i0 % 128, "
                      "j0 % 128, ldc % 4 and alignment required");
        return MXLU_E_NOMEM;
    }
    Lq += (size_t)i0 * BK8;   // line i0 (j0) of every K chunk
    Uq += (size_t)j0 * BK8;
    sLx += i0;                // sLx[b Mp + r], sUx[b Np + c]: line i0 (j0) of every block
    sUx += j0;
    const int64_t tiles_m = (M + kTm8 - 1) / kTm8, tiles_n = (N + kTn8 - 1) / kTn8;
    const dim3 grid((unsigned)(tiles_m * tiles_n));
    const float *none = nullptr;
    if (fmt == kFmtBf16)
        hipLaunchKernelGGL((lp_schur8_kernel<kFmtBf16, 2, true>), grid, dim3(256), 0, s, M, N, K,
                           Lq, Mp, none, Uq, Np, none, 4, sLx, sUx, C, ldc, (int)tiles_m,
                           (int)tiles_n);
    else
        hipLaunchKernelGGL((lp_schur8_kernel<kFmtFp16, 2, true>), grid, dim3(256), 0, s, M, N, K,
                           Lq, Mp, none, Uq, Np, none, 4, sLx, sUx, C, ldc, (int)tiles_m,
                           (int)tiles_n);
    MXLU_LAUNCH_CHECK();
    return 0;
}

}  // namespace mxlu
