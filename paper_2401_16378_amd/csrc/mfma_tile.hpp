// Device building blocks of the matrix-core path, shared by the
// single-matrix kernels (mfma.hip) and the persistent uneven-batch kernel
// (batched.hip).
#pragma once
//
// Matrix-core (MFMA) path for gfx950: the paper's O(2^N)-per-coefficient
// sum (Eq. (c_def_in_terms_of_fn)) for all coefficients at once, i.e. the
// O(8^N) total of section 3, evaluated as a dense contraction
//
//     C[p][x] = sum_q H[p][q] * In[q][x],      H[p][q] = (-1)^{popc(p & q)}
//
// forward (decomposition):  q = i, p = z, In[i][x] = G[i^x][i] (the gathered
//   XOR diagonal v_x), out[n(x,z)] = 2^-N (-i)^{popc(x&z)} C[z][x];
// adjoint (recomposition / gradient):  q = z, p = i,
//   In[z][x] = i^{popc(x&z)} c[n(x,z)],  G[i^x][i] = scale * C[i][x].
//
// Two kernels.
//
// pack: an HBM-bound pass that gathers In (the XOR diagonals of G, or the
//   phased coefficient blocks), converts it to the matrix-core operand
//   format and stores it in the exact lane order of the MFMA B operand, one
//   contiguous 1 KiB fragment (64 lanes x 16 bytes) per (32 flip masks,
//   16 or 8 K values, plane, re/im).  A thread owns an aligned 4x4
//   micro-block: 4 rows x 4 columns of G, which the XOR map sends to 4 flip
//   masks x 4 consecutive q, or 16 consecutive coefficients, which form a
//   4x4 (z,x) block; the block is transposed through LDS so every global
//   store is a full 1 KiB fragment.
//
// contract: each wave owns RB*32 rows p and 32 flip masks x (64 real B
//   columns: re, then im) and walks the whole K range, streaming its B
//   fragments from L2 through a register ring PF slices deep.  H is the
//   Sylvester-Hadamard sign matrix: every entry is +-1, exact in any format,
//   so it never touches memory; over an aligned 32-row block it is one fixed
//   32x32 block times a sign fixed by the blocks' high bits, and the kernel
//   keeps that block's fragments and their negations in registers, choosing
//   among them at compile time plus one uniform sign per group of slices.
//   No LDS and no barrier in the main loop; the epilogue stages each 32x32
//   output block in LDS so it leaves as one contiguous run of coefficients
//   (forward) or one aligned 32x32 square of G (adjoint).
//
// Precision.  PLANES = 3: each binary32 component g is split as
// g ~ hi + mid + lo (three bf16 numbers, hi on a power-of-two grid shared by
// the 4x4 micro-block, see split3); bf16 MFMA accumulates hi into one FP32
// accumulator, where the sums stay exact, and mid + lo into a second, and the
// two are added in binary64 in the epilogue before the phase and scale.
// PLANES = 2: the matrix is first multiplied by a power of two 2^pe that
// brings its largest component just below 2^15 (a reduction pass finds it),
// then each component is split as g ~ hi + 2^-11 lo (two fp16 numbers, hi
// with 11 significant bits on the micro-block grid, see split2); fp16 MFMA
// accumulates each plane into its own FP32 accumulator and the epilogue
// forms hi + 2^-11 lo in binary64 and undoes 2^pe with the scale.
// PLANES = 1: binary32 MFMA on the binary32 components.
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pauli {
namespace mfma {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int XT = 32;       // flip masks per fragment column block
constexpr int FRAG = 1024;   // bytes per B fragment (64 lanes x 16 bytes)

__device__ inline uint32_t pack_bf16(float a, float b) {
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ inline float lo_half(uint32_t u) { return __builtin_bit_cast(float, u << 16); }
__device__ inline float hi_half(uint32_t u) { return __builtin_bit_cast(float, u & 0xFFFF0000u); }
__device__ inline uint32_t pack_f16(float a, float b) {
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}

// Bits of +1 in the 16-bit operand format of the split (bf16 for three
// planes, fp16 for two); setting bit 15 negates.
template <int PLANES>
constexpr uint32_t ONE16 = PLANES == 2 ? 0x3C00u : 0x3F80u;

// One 32x32x16 MFMA step of a 16-bit plane, operands given as raw bits.
template <int PLANES>
__device__ inline f32x16 mfma16(const u32x4& a, const u32x4& b, const f32x16& c) {
    if constexpr (PLANES == 2)
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
}

// Three-way bf16 split of two binary32 values a, b against a power-of-two
// grid u (with inv_u = 1/u, both exact):
//   hi  = u * rint(x / u)        (|x| < 256 u, so hi has <= 8 significant bits
//                                 and is exact in bf16)
//   mid = bf16(x - hi),  lo = bf16(x - hi - mid)
// x - hi and x - hi - mid are exact in binary32, so hi + mid + lo carries
// every bit of x except at most those below 2^-17 |x - hi|.  All hi terms of
// a micro-block are multiples of the same u, which keeps the FP32 sums of hi
// terms exact over the whole K range for any input whose partial sums stay
// below 2^24 times the smallest grid (about 2^16 times the smallest block
// maximum), instead of rounding away the low bits of small terms.
__device__ inline void split3(float a, float b, float u, float inv_u, uint32_t& h, uint32_t& m,
                              uint32_t& l) {
    const float ha = __builtin_rintf(a * inv_u) * u, hb = __builtin_rintf(b * inv_u) * u;
    h = pack_bf16(ha, hb);
    const float ra = a - ha, rb = b - hb;
    m = pack_bf16(ra, rb);
    const float qa = ra - lo_half(m), qb = rb - hi_half(m);
    l = pack_bf16(qa, qb);
}

// Grid of a micro-block: u = 2^(e-8) for the exponent e with max|x| < 2^e,
// clamped so that u and 1/u stay normal binary32 numbers.
__device__ inline void block_grid(float maxabs, float& u, float& inv_u) {
    int e = (int)((__builtin_bit_cast(uint32_t, maxabs) >> 23) & 0xFFu) - 126;
    e = e < -110 ? -110 : (e > 120 ? 120 : e);
    u = __builtin_bit_cast(float, (uint32_t)(127 + e - 8) << 23);
    inv_u = __builtin_bit_cast(float, (uint32_t)(127 - e + 8) << 23);
}

// Two-way fp16 split of two prescaled binary32 values a, b against the
// micro-block grid u (|x| < 2^11 u, 2^-24 <= u <= 2^4, inv_u = 1/u):
//   hi = u * rint(x / u)          an integer of at most 11 bits times u, so
//                                 exact in fp16 (|hi| <= 2^15)
//   lo = fp16(2^11 (x - hi))      x - hi is exact in binary32, |x - hi| <= u/2
// hi + 2^-11 lo equals x to within 2^-12 |x - hi| <= 2^-13 u, i.e. about
// 2^-24 of the block's largest component.  As for split3, every hi term is a
// multiple of its block's grid, so the FP32 sums of hi terms are exact while
// they stay below 2^24 times the smallest grid.
__device__ inline void split2(float a, float b, float u, float inv_u, uint32_t& h, uint32_t& l) {
    const float ha = __builtin_rintf(a * inv_u) * u, hb = __builtin_rintf(b * inv_u) * u;
    h = pack_f16(ha, hb);
    l = pack_f16((a - ha) * 2048.f, (b - hb) * 2048.f);
}

// Grid of a micro-block for split2: u = 2^(e-11) for the exponent e with
// max|x| < 2^e, at least 2^-24 (the smallest fp16 step).
__device__ inline void block_grid16(float maxabs, float& u, float& inv_u) {
    int e = (int)((__builtin_bit_cast(uint32_t, maxabs) >> 23) & 0xFFu) - 126;
    e = e < -13 ? -13 : e;
    u = __builtin_bit_cast(float, (uint32_t)(127 + e - 11) << 23);
    inv_u = __builtin_bit_cast(float, (uint32_t)(127 - e + 11) << 23);
}

// Prescale exponent of the two-plane split for a matrix whose largest
// component (in absolute value, as binary32) is maxabs: pe = 15 - e with
// maxabs < 2^e, so that 2^pe maxabs < 2^15.
__host__ __device__ inline int prescale_exponent(float maxabs) {
    const int e = (int)((__builtin_bit_cast(uint32_t, maxabs) >> 23) & 0xFFu) - 126;
    return 15 - e;
}

// Largest of m over a 256-thread workgroup (red: 4 floats of LDS); every
// thread gets the result.
__device__ inline float block_max256(float m, float* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = __builtin_fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    return __builtin_fmaxf(__builtin_fmaxf(red[0], red[1]), __builtin_fmaxf(red[2], red[3]));
}

template <bool IN128>
__device__ inline f32x2 load_elem(const unsigned char* base, size_t idx) {
    if constexpr (IN128) {
        const double2 v = ((const double2*)base)[idx];
        return f32x2{(float)v.x, (float)v.y};
    } else {
        const float2 v = ((const float2*)base)[idx];
        return f32x2{v.x, v.y};
    }
}

// ---------------------------------------------------------------------------
// Packed operand layout, per matrix, with Dp = max(2^N, 32):
//   16-bit planes (P = 3 bf16 or P = 2 fp16): fragment (xb, s, pl, cb) at
//         ((xb * Dp/16 + s) * 2P + pl * 2 + cb) KiB,
//         lane l = x_l + 32h holds K = 16s + 8h + j, j < 8, of column x_l;
//   fp32: fragment (xb, s, cb) at ((xb * Dp/8 + s) * 2 + cb) KiB,
//         lane l holds K = 8s + 4h + t, t < 4.
// pl = hi/mid/lo (or hi/lo) plane, cb = 0 real parts, 1 imaginary parts.
// ---------------------------------------------------------------------------
template <int PLANES>
struct Pack {
    static_assert(PLANES >= 1 && PLANES <= 3, "one, two or three planes");
    static constexpr int SK = PLANES == 1 ? 8 : 16;        // K per slice
    static constexpr int LOG_SK = PLANES == 1 ? 3 : 4;
    static constexpr int NPL = 2 * PLANES;                 // fragments per slice
    static constexpr int ESZ = PLANES == 1 ? 4 : 2;        // bytes per element
    static constexpr int SLICE_BYTES = NPL * FRAG;
    static constexpr int EB = NPL * ESZ;                   // packed bytes per matrix element
    static constexpr int ACC = PLANES == 1 ? 1 : 2;        // FP32 accumulators per output
};

constexpr int slice_k(int planes) { return planes == 1 ? 8 : 16; }

__host__ __device__ inline uint32_t padded_dim(int N) { return N < 5 ? 32u : (1u << N); }

constexpr int PACK_KT = 128;   // K per pack workgroup (less when Dp < 128)

// Adjoint pack: a wave's 32 x 32 block of coefficients staged in LDS as
// binary32 pairs, 16 bytes of padding after every 16 entries (the per-thread
// reads of 16 consecutive entries then fall in distinct banks).
constexpr int ADJ_STAGE = 1024 + 2 * 64;   // f32x2 per wave

template <int PLANES, int DIR = FORWARD>
constexpr int pack_lds_bytes() {
    const int stage = Pack<PLANES>::NPL * XT * (PACK_KT * Pack<PLANES>::ESZ + 16);
    const int adj = 4 * ADJ_STAGE * 8;
    return DIR == FORWARD || stage >= adj ? stage : adj;
}

__host__ __device__ inline uint32_t pack_tiles(int N) {
    const uint32_t Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)PACK_KT ? Dp : (uint32_t)PACK_KT;
    return (Dp / XT) * (Dp / KT);
}

// Hermitian forward pack: tiles of flip masks X0 >= hmin (hmin >= 128, a
// power of two no smaller than the contraction's half-walk threshold) whose
// K range has the top bit of X0 set are never read by the half walk, so they
// are not packed.  All 128 K values of a tile share that bit, so exactly half
// of the tiles of such a 32-mask slab remain.  The pack grid holds only the
// remaining tiles: herm_pack_tiles(N, hmin) of them, block t packing tile
// herm_pack_tile(N, hmin, t) of pack_tiles(N), in increasing order.
static_assert(PACK_KT == 128, "the tiles of a slab split on bit 7 and above of K");

__host__ __device__ inline uint32_t herm_pack_tiles(int N, uint32_t hmin) {
    const uint32_t Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)PACK_KT ? Dp : (uint32_t)PACK_KT;
    const uint32_t nKT = Dp / KT, nXB = Dp / XT;
    const uint32_t whole = nXB < hmin / XT ? nXB : hmin / XT;   // slabs packed whole
    return whole * nKT + (nXB - whole) * (nKT / 2);
}

__device__ inline uint32_t herm_pack_tile(int N, uint32_t hmin, uint32_t t) {
    const uint32_t Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)PACK_KT ? Dp : (uint32_t)PACK_KT;
    const uint32_t nKT = Dp / KT, nXB = Dp / XT;
    const uint32_t whole = nXB < hmin / XT ? nXB : hmin / XT;
    if (t < whole * nKT) return t;
    // a half slab (then Dp > hmin >= 128, so KT = 128 and nKT >= 2): the j-th
    // K tile whose bit b = log2(X0) - 7 is clear
    const uint32_t u = t - whole * nKT, half = nKT / 2;
    const uint32_t xb = whole + u / half, j = u % half;
    const uint32_t b = 31u - (uint32_t)__builtin_clz(xb * XT) - 7u;
    const uint32_t kt = ((j >> b) << (b + 1)) | (j & ((1u << b) - 1u));
    return xb * nKT + kt;
}

// Split one thread's 4x4 micro-block v (forward: v[a * 4 + b] = G[row a][col
// b]; adjoint: 16 consecutive phased coefficients) into the operand format
// and store it in the LDS staging tile at flip-mask group xh (x_l / 4) and K
// slot kh: plane-major, 32 flip masks per plane, pitch bytes per mask.
// pe: the prescale exponent of the two-plane split (unused otherwise).
template <int PLANES, int DIR>
__device__ __attribute__((always_inline)) inline void stage_block(f32x2 (&v)[16], int xh, int kh, int pe,
                                                                  unsigned char* lds, uint32_t pitch) {
    using P = Pack<PLANES>;
    float gu = 1.f, ginv = 1.f;
    if constexpr (PLANES == 2) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
            v[r] = f32x2{__builtin_ldexpf(v[r].x, pe), __builtin_ldexpf(v[r].y, pe)};
    }
    if constexpr (PLANES >= 2) {
        float mx = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r)
            mx = __builtin_fmaxf(mx, __builtin_fmaxf(__builtin_fabsf(v[r].x), __builtin_fabsf(v[r].y)));
        if constexpr (PLANES == 3) block_grid(mx, gu, ginv);
        else block_grid16(mx, gu, ginv);
    }
#pragma unroll
    for (int x2 = 0; x2 < 4; ++x2) {
        f32x2 e[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if constexpr (DIR == FORWARD) {
                e[b] = v[((x2 ^ b) << 2) | b];  // row a = x2 ^ b, column b
            } else {
                const int d = x2 ^ b;             // (x ^ z) low bits
                e[b] = v[(d & 1) | ((b & 1) << 1) | ((d >> 1) << 2) | ((b >> 1) << 3)];
            }
        }
        unsigned char* cbase = lds + (xh * 4 + x2) * pitch + kh * P::ESZ;
        const uint32_t PS = XT * pitch;  // plane stride
        if constexpr (PLANES == 3) {
            uint32_t hr0, mr0, lr0, hr1, mr1, lr1, hi0, mi0, li0, hi1, mi1, li1;
            split3(e[0].x, e[1].x, gu, ginv, hr0, mr0, lr0);
            split3(e[2].x, e[3].x, gu, ginv, hr1, mr1, lr1);
            split3(e[0].y, e[1].y, gu, ginv, hi0, mi0, li0);
            split3(e[2].y, e[3].y, gu, ginv, hi1, mi1, li1);
            *(u32x2*)(cbase + 0 * PS) = u32x2{hr0, hr1};
            *(u32x2*)(cbase + 1 * PS) = u32x2{hi0, hi1};
            *(u32x2*)(cbase + 2 * PS) = u32x2{mr0, mr1};
            *(u32x2*)(cbase + 3 * PS) = u32x2{mi0, mi1};
            *(u32x2*)(cbase + 4 * PS) = u32x2{lr0, lr1};
            *(u32x2*)(cbase + 5 * PS) = u32x2{li0, li1};
        } else if constexpr (PLANES == 2) {
            uint32_t hr0, lr0, hr1, lr1, hi0, li0, hi1, li1;
            split2(e[0].x, e[1].x, gu, ginv, hr0, lr0);
            split2(e[2].x, e[3].x, gu, ginv, hr1, lr1);
            split2(e[0].y, e[1].y, gu, ginv, hi0, li0);
            split2(e[2].y, e[3].y, gu, ginv, hi1, li1);
            *(u32x2*)(cbase + 0 * PS) = u32x2{hr0, hr1};
            *(u32x2*)(cbase + 1 * PS) = u32x2{hi0, hi1};
            *(u32x2*)(cbase + 2 * PS) = u32x2{lr0, lr1};
            *(u32x2*)(cbase + 3 * PS) = u32x2{li0, li1};
        } else {
            *(f32x4*)(cbase) = f32x4{e[0].x, e[1].x, e[2].x, e[3].x};
            *(f32x4*)(cbase + PS) = f32x4{e[0].y, e[1].y, e[2].y, e[3].y};
        }
    }
}

// The 4x4 micro-block of G that thread (square g, block w6) of a pack tile
// with flip masks X0.. and K values Q0.. gathers: rows ((Q0 + 32 g) ^ X0) &
// ~31 + 4 (w6 >> 3) .., columns Q0 + 32 g + 4 (w6 & 7) .., zero outside a
// matrix of order D < 32 (`full`: D >= 32).  Returns its staging slots.
template <bool IN128>
__device__ __attribute__((always_inline)) inline void load_block_fwd(const unsigned char* __restrict__ src, uint32_t D,
                                                                     bool full, uint32_t X0, uint32_t Q0, int g, int w6,
                                                                     f32x2 (&v)[16], int& xh, int& kh) {
    const int mr = w6 >> 3, mc = w6 & 7;
    const uint32_t q0 = Q0 + 32 * g + 4 * mc;
    const uint32_t r0 = (((Q0 + 32 * g) ^ X0) & ~31u) + 4 * mr;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t r = r0 + a, q = q0 + b;
            v[a * 4 + b] = (full || (r < D && q < D)) ? load_elem<IN128>(src, (size_t)r * D + q) : f32x2{0.f, 0.f};
        }
    xh = mr ^ mc;
    kh = 32 * g + 4 * mc;
}

// Pack tile t (of pack_tiles(N)) of one matrix: 32 flip masks x KT values of
// q.  256 threads; src = the matrix (or coefficient vector), ws = its packed
// operand; lds holds pack_lds_bytes<PLANES, DIR>() bytes.
// pe: the prescale exponent of the two-plane split (unused otherwise).
template <int PLANES, int DIR, bool IN128>
__device__ inline void pack_tile(const unsigned char* __restrict__ src, unsigned char* __restrict__ ws,
                                 int N, uint32_t t, unsigned char* lds, int pe = 0) {
    using P = Pack<PLANES>;
    const uint32_t D = 1u << N, Dp = padded_dim(N);
    const uint32_t KT = Dp < (uint32_t)PACK_KT ? Dp : (uint32_t)PACK_KT;
    const uint32_t pitch = KT * P::ESZ + 16;
    const uint32_t nKT = Dp / KT;
    const uint32_t xb = t / nKT, kt = t % nKT;
    const uint32_t X0 = xb * XT, Q0 = kt * KT;
    const bool full = D >= 32u;
    const int tid = threadIdx.x;
    const bool active = (uint32_t)tid < 2 * KT;
    const int g = tid >> 6, w6 = tid & 63;       // 32x32 square g, block w6 in it
    f32x2 v[16];

    if constexpr (DIR != FORWARD) {
        // The 32 x 32 coefficients of square g are 1024 consecutive entries
        // of the vector.  Read them lane-consecutive (each load instruction
        // covers 64 neighbouring entries) into the wave's LDS block, then take
        // each thread's 16 consecutive entries from there.  `full` is uniform.
        if (full) {
            f32x2* blk = (f32x2*)lds + g * ADJ_STAGE;
            const uint32_t nb = pauli_index(X0, Q0 + 32 * g);
            if (active) {
                f32x2 c[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) c[i] = load_elem<IN128>(src, nb + 64 * i + w6);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int o = 64 * i + w6;
                    blk[o + 2 * (o >> 4)] = c[i];
                }
            }
            __syncthreads();
            if (active) {
                const f32x4* b4 = (const f32x4*)(blk + 18 * w6);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const f32x4 q = b4[j];
                    v[2 * j] = f32x2{q.x, q.y};
                    v[2 * j + 1] = f32x2{q.z, q.w};
                }
            }
            __syncthreads();   // the staging below overwrites the LDS
        }
    }

    // one 4x4 micro-block per thread: 2*KT of them in the 32 x KT tile
    if (active) {
        int xh, kh;                              // column group (x_l / 4), first K slot
        if constexpr (DIR == FORWARD) {
            load_block_fwd<IN128>(src, D, full, X0, Q0, g, w6, v, xh, kh);
        } else {
            const uint32_t zb = Q0 + 32 * g;
            const uint32_t nb = pauli_index(X0, zb);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t o = 16 * w6 + r;
                const uint32_t zl = compact_even(o >> 1), xl = compact_even(o) ^ zl;
                const uint32_t z = zb + zl, x = X0 + xl;
                f32x2 c = {0.f, 0.f};
                if (full) c = v[r];
                else if (z < D && x < D) c = load_elem<IN128>(src, nb + o);
                float re = c.x, im = c.y;
                rotate_minus_i(re, im, 3u * (uint32_t)__popc(x & z));  // i^{popc(x&z)}
                v[r] = f32x2{re, im};
            }
            // 16 consecutive coefficients o = 16*w6 + r, r = (x^z)_0 | z_0<<1 | (x^z)_1<<2 | z_1<<3
            const uint32_t o = 16 * w6;
            const int zl = compact_even(o >> 1), xl = compact_even(o) ^ zl;
            xh = xl >> 2;
            kh = 32 * g + zl;
        }
        stage_block<PLANES, DIR>(v, xh, kh, pe, lds, pitch);
    }
    __syncthreads();

    // Write whole fragments: KT/SK slices x NPL fragments, 64 lanes x 16 bytes.
    const int lane = tid & 63, wave = tid >> 6;
    const int xl = lane & 31, h = lane >> 5;
    const uint32_t nfrag = (KT / P::SK) * P::NPL;
    unsigned char* dst = ws + ((size_t)xb * (Dp / P::SK) + Q0 / P::SK) * P::SLICE_BYTES;
    for (uint32_t f = wave; f < nfrag; f += 4) {
        const uint32_t s = f / P::NPL, pl = f % P::NPL;
        const unsigned char* srcl = lds + pl * XT * pitch + xl * pitch + (s * P::SK + h * (P::SK / 2)) * P::ESZ;
        *(u32x4*)(dst + (size_t)f * FRAG + lane * 16) = *(const u32x4*)srcl;
    }
}

// Slices per unrolled step of the register-ring contraction: twice the
// larger of the sign group (32*RB K values) and the ring depth.
constexpr int ring_step_slices(int planes, int rb, int pf) {
    const int u = 32 * rb / slice_k(planes);
    return 2 * (u > pf ? u : pf);
}

// First flip mask X0 (a multiple of 32) from which the Hermitian contraction
// of a register-ring tile walks half of K: X0 >= (step length) * (K per slice).
constexpr uint32_t herm_half_from(int planes, int rb, int pf) {
    return (uint32_t)ring_step_slices(planes, rb, pf) * (uint32_t)slice_k(planes);
}

// Hermitian tiles that also halve the rows: a half walk (X0 >= hf) whose
// skipped bit 2^b (the top bit of X0) spans whole workgroup tiles of mt rows,
// when the LDS holds two output stages of `waves` x 1024 coefficients.
constexpr uint32_t LDS_BYTES_MAX = 160u * 1024u;
__host__ __device__ constexpr bool herm_pair_stage_fits(int waves, int out128) {
    return (uint32_t)waves * 2u * 1024u * (out128 ? 16u : 8u) <= LDS_BYTES_MAX;
}
__host__ __device__ inline bool herm_pair_rows(uint32_t X0, uint32_t hf, uint32_t mt, int waves, int out128) {
    return X0 >= hf && X0 != 0 && (1u << (31 - __builtin_clz(X0))) >= mt && herm_pair_stage_fits(waves, out128);
}

// Binary32 plane: an MFMA accumulator chain adds at most FLUSH_SLICES slices
// (256 K values) before it is added into a running binary32 total and
// restarted from zero.  The boundary is a fixed K offset, the same for every
// tile shape, so all tiles still sum each output in one order; a chain of 256
// terms instead of 2^N cuts the accumulated rounding by about sqrt(2^N / 256).
constexpr uint32_t FLUSH_SLICES = 256 / Pack<1>::SK;

// Register-ring tiles of 4 x 32 rows per wave need the 128 accumulators plus
// the 128-register binary32 total next to the fragment ring, more than the
// register file holds; compiled that way they spill and the adjoint direction
// returned wrong values, so the binary32 plane does not offer them (its
// LDS-staged and 2 x 32-row tiles run at the same speed).
constexpr bool ring_tile_ok(int planes, int rb) { return !(planes == 1 && rb == 4); }

template <int RB>
__device__ inline void flush_into(f32x16 (&tot)[1][RB][2], f32x16 (&acc)[1][RB][2]) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                tot[0][rb][cb][r] += acc[0][rb][cb][r];
                acc[0][rb][cb][r] = 0.f;
            }
}

// Epilogue shared by the contraction variants: binary64 recombination of the
// accumulators, phase, scale, and an LDS-staged store of each 32x32 block as
// one contiguous coefficient run (forward) or one aligned square of G
// (adjoint).  lds holds WAVES * 1024 * esz bytes; all waves of the
// workgroup must call it (it contains barriers).  HERM (forward only): the
// input is Hermitian, so the sum is real when popc(x&z) is even and
// imaginary when it is odd; the other component, zero in exact arithmetic,
// is dropped before the phase, which leaves every coefficient exactly real.
// HERM with HF > 0: a tile of MT rows whose flip masks start at X0 >= HF was
// a half walk over K (bit b = the top bit of X0 skipped); when 2^b >= MT (and
// the workgroup's LDS has room for a second stage) the rows Pw ^ 2^b hold the
// same sums, so each value is staged a second time for them, with the other
// component (the parity of popc(x&z) flips), and both runs are stored.  The
// condition is re-derived here from X0 rather than carried through the
// contraction in a register.
template <int PLANES, int RB, int DIR, bool HERM = false, uint32_t HF = 0, uint32_t MT = 0>
__device__ __attribute__((always_inline)) inline void store_tile(const f32x16 (&acc)[Pack<PLANES>::ACC][RB][2], unsigned char* __restrict__ dst,
                                  int N, uint32_t X0, uint32_t Pw, double scale, int out128, unsigned char* lds) {
    uint32_t pair = 0;
    if constexpr (HERM && HF > 0) {
        if (herm_pair_rows(X0, HF, MT, (int)(MT / (32 * RB)), out128)) pair = 1u << (31 - __builtin_clz(X0));
    }
    constexpr int ACC = Pack<PLANES>::ACC;
    constexpr double LOW = PLANES == 2 ? 1.0 / 2048.0 : 1.0;   // weight of the second accumulator
    const uint32_t D = 1u << N;
    // The thread index passes through an empty asm statement, so that the
    // staging addresses derived from it are formed here, at each call, and
    // not hoisted by the compiler into registers held across the contraction
    // (in the persistent kernel's tile loop they would otherwise stay live
    // next to the accumulators and spill).
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const int esz = out128 ? 16 : 8;
    unsigned char* stage = lds + wave * 1024 * esz;
    // the partner rows' stage, after the WAVES stages (allocated only where pairing can happen)
    unsigned char* stage2 = HERM && HF > 0 ? lds + (MT / (32 * RB) + wave) * 1024 * esz : stage;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const uint32_t pb = Pw + 32 * rb;   // first row of this 32x32 block
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t pl = 8 * (r >> 2) + 4 * h + (r & 3);
            double re = (double)acc[0][rb][0][r];
            double im = (double)acc[0][rb][1][r];
            if constexpr (ACC == 2) {
                re += LOW * (double)acc[ACC - 1][rb][0][r];
                im += LOW * (double)acc[ACC - 1][rb][1][r];
            }
            re *= scale;
            im *= scale;
            uint32_t slot;
            if constexpr (DIR == FORWARD) {
                const uint32_t ny = (uint32_t)__popc((X0 + l32) & (pb + pl));
                slot = pauli_index((uint32_t)l32, pl);           // offset inside the 1024-run
                if constexpr (HERM) {
                    double qr = re, qi = im;                      // row pb + pl ^ pair: the other component
                    if (ny & 1) {
                        re = 0.0;
                        qi = 0.0;
                    } else {
                        im = 0.0;
                        qr = 0.0;
                    }
                    if (pair) {
                        rotate_minus_i(qr, qi, ny + 1u);
                        if (out128) *(double2*)(stage2 + slot * 16) = make_double2(qr, qi);
                        else *(float2*)(stage2 + slot * 8) = make_float2((float)qr, (float)qi);
                    }
                }
                rotate_minus_i(re, im, ny);
            } else {
                slot = ((pl ^ (uint32_t)l32) << 5) | pl;        // (row, col) inside the 32x32 square
            }
            if (out128) *(double2*)(stage + slot * 16) = make_double2(re, im);
            else *(float2*)(stage + slot * 8) = make_float2((float)re, (float)im);
        }
        __syncthreads();
        if constexpr (DIR == FORWARD) {
            // contiguous run of min(1024, 4^N) coefficients starting at n(X0, pb)
            const uint32_t run = D < 32u ? D * D : 1024u;
            unsigned char* o = dst + (size_t)pauli_index(X0, pb) * esz;
            if (pb < D) {
                if (run * esz >= 16) {
                    for (uint32_t b = lane * 16; b < run * esz; b += 64 * 16)
                        *(u32x4*)(o + b) = *(const u32x4*)(stage + b);
                } else if (lane == 0) {
                    *(u32x2*)o = *(const u32x2*)stage;   // N = 0, binary32 output
                }
            }
            if constexpr (HERM) {
                if (pair) {   // 1024-runs only: 2^b >= MT >= 32 rows, so N >= 6
                    unsigned char* o2 = dst + (size_t)pauli_index(X0, pb ^ pair) * esz;
                    for (uint32_t b = lane * 16; b < run * esz; b += 64 * 16)
                        *(u32x4*)(o2 + b) = *(const u32x4*)(stage2 + b);
                }
            }
        } else {
            // 32x32 square of G: rows (pb ^ X0) + rl, columns pb + cl
            const uint32_t w = D < 32u ? D : 32u;
            const uint32_t rowbytes = w * esz;
            const uint32_t r0 = (pb ^ X0) & ~31u;
            if (pb < D) {
                if (rowbytes >= 16) {
                    for (uint32_t b = lane * 16; b < w * rowbytes; b += 64 * 16) {
                        const uint32_t rl = b / rowbytes, cb = b % rowbytes;
                        *(u32x4*)(dst + ((size_t)(r0 + rl) * D + pb) * esz + cb) =
                            *(const u32x4*)(stage + rl * 32 * esz + cb);
                    }
                } else if (lane == 0) {
                    *(u32x2*)dst = *(const u32x2*)stage;     // N = 0, binary32 output
                }
            }
        }
        __syncthreads();
    }
}

// One output tile: flip masks xb*32.., rows mb*MT.. (MT = WAVES*RB*32) of a
// matrix with padded order Dp.  Waves whose rows lie beyond Dp (only when
// Dp < MT) skip the contraction but take part in the epilogue barriers.
// wsm = the matrix's packed operand, dst = its output; lds holds
// WAVES * 1024 * esz bytes of staging.
//
// HERM (forward, Hermitian G): v_x[i ^ x] = conj(v_x[i]) and
// (-1)^{popc((i^x)&z)} = (-1)^{popc(i&z)} (-1)^{popc(x&z)}, so the sum over
// the pair {i, i^x} is s_i (v + conj v) = 2 s_i Re v when popc(x&z) is even
// and s_i (v - conj v) = 2i s_i Im v when it is odd: the sum over the i
// with one bit b of i clear, doubled, gives the whole sum, provided every
// flip mask of the tile has bit b set.  The tile's flip masks X0..X0+31
// (X0 = 32 xb) share the bits of X0; with b the top bit of X0 and
// X0 >= GS*SK, the skipped bit of the slice index lies above the unrolled
// step, so each step still walks GS (or GSL) consecutive slices with the
// same compile-time sign pattern, half as many steps.  Tiles with smaller X0
// walk the whole K range (the same result without the shortcut).
template <int PLANES, int RB, int WAVES, int DIR, int PF, bool HERM = false>
__device__ __attribute__((always_inline)) inline void contract_tile(const unsigned char* __restrict__ wsm, unsigned char* __restrict__ dst,
                                     int N, uint32_t xb, uint32_t mb, double scale, int out128,
                                     unsigned char* lds) {
    using P = Pack<PLANES>;
    constexpr int ACC = P::ACC;
    constexpr int MT = WAVES * RB * 32;                    // rows per workgroup
    constexpr int U = 32 * RB / P::SK;                     // slices per sign group (32*RB K)
    constexpr int GS = ring_step_slices(PLANES, RB, PF);   // slices per unrolled step
    static_assert(GS % U == 0 && GS % PF == 0, "ring depth and sign group must nest");
    static_assert(!HERM || DIR == FORWARD, "the Hermitian shortcut is a forward-only property");

    const uint32_t Dp = padded_dim(N);
    const uint32_t nS = Dp / P::SK;
    const uint32_t X0 = xb * XT;

    // Slices walked (nK) and the map from the walk index to the slice index
    // (a zero inserted at bit beta) when only half of K is summed.
    uint32_t nK = nS, beta = 0;
    bool half = false;
    if constexpr (HERM) {
        if (X0 >= herm_half_from(PLANES, RB, PF)) {
            half = true;
            const uint32_t tb = (uint32_t)(31 - __builtin_clz(X0));   // bit b, set in every flip mask of the tile
            beta = tb - (uint32_t)P::LOG_SK;
            nK = nS >> 1;
            // The half walk never reads bit b of i, so rows z and z ^ 2^b get
            // the same sums; the tile with bit b of its rows clear stores both
            // (store_tile), and the tile with it set has nothing left to do.
            if (herm_pair_rows(X0, herm_half_from(PLANES, RB, PF), (uint32_t)MT, WAVES, out128) &&
                (((mb * (uint32_t)MT) >> tb) & 1u))
                return;
        }
    }
    auto slice_of = [&](uint32_t c) -> uint32_t {
        if constexpr (HERM) {
            const uint32_t low = (1u << beta) - 1u;
            return half ? (((c & ~low) << 1) | (c & low)) : c;
        } else {
            return c;
        }
    };
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));   // per call, as in store_tile
    const int lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const uint32_t Pw = mb * MT + wave * RB * 32;          // first row of this wave
    const unsigned char* wsx = wsm + (size_t)xb * nS * P::SLICE_BYTES + lane * 16;

    // ---- sign fragments of the 32x32 Sylvester block ----
    // 16-bit: lane (row p_l = l32, half h) holds K slots q_l = 16e + 8h + j, j < 8,
    //       for the two 16-wide slices e of a 32-wide block.
    // fp32: lane holds q_l = 8e + 4h + t for slice e < 4, step t < 4.
    uint32_t fA[2][4];   // 16-bit pairs, [e][j/2]
    float fF[4][4];      // fp32, [e][t]
    if constexpr (PLANES >= 2) {
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t q0 = 16 * e + 8 * h + 2 * jj;
                const uint32_t s0 = ONE16<PLANES> | ((__popc(l32 & q0) & 1) ? 0x8000u : 0u);
                const uint32_t s1 = ONE16<PLANES> | ((__popc(l32 & (q0 + 1)) & 1) ? 0x8000u : 0u);
                fA[e][jj] = s0 | (s1 << 16);
            }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                fF[e][t] = (__popc(l32 & (8 * e + 4 * h + t)) & 1) ? -1.f : 1.f;
    }

    f32x16 acc[ACC][RB][2], tot[1][RB][2];   // tot: binary32 plane's flushed total
#pragma unroll
    for (int a = 0; a < ACC; ++a)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][rb][cb][r] = tot[0][rb][cb][r] = 0.f;

    // ---- B fragment ring ----
    u32x4 ring[PF][P::NPL];
    auto fetch = [&](int slot, uint32_t s) {
        const unsigned char* p = wsx + (size_t)s * P::SLICE_BYTES;
#pragma unroll
        for (int f = 0; f < P::NPL; ++f) ring[slot][f] = *(const u32x4*)(p + f * FRAG);
    };
    const bool active = Pw < Dp;                 // idle waves skip the contraction
    // Main loop: GSX slices per unrolled step (the ring and the sign groups
    // both nest in it).  The forward bf16 tiles of 4 x 32 rows per wave also
    // get a step four times longer when the K length allows it: the compiler waits
    // for every outstanding fragment load at the top of each step, and a
    // longer step does that less often (measured 1.7% at N = 14); the sum
    // order, and so the result, is the same for both step lengths.
    auto main_loop = [&](auto gs_tag) {
    constexpr int GSX = decltype(gs_tag)::value;
#pragma unroll
    for (int k = 0; k < PF; ++k) fetch(k, slice_of((uint32_t)k < nK ? k : nK - 1));

    u32x4 Ap[2], An[2];
    float ts = 1.f;
    for (uint32_t s0 = 0; s0 < nK; s0 += GSX) {
        const uint32_t sr = slice_of(s0);   // the step's GSX slices are sr, sr+1, ...
        // first slice of the next step (the refills of this step's last PF
        // slots read it and its successors); after the last step the refills
        // are never used and reread this step's slices
        const uint32_t sn = s0 + GSX < nK ? slice_of(s0 + GSX) : sr;
#pragma unroll
        for (int uu = 0; uu < GSX; ++uu) {
            const int u = uu % U, slot = uu % PF;
            if (u == 0) {
                // sign of this wave's rows against this group of 32*RB K values
                const bool neg_grp = __popc((Pw >> 5) & (((sr + uu) * P::SK) >> 5)) & 1;
                if constexpr (PLANES >= 2) {
                    const uint32_t tm = neg_grp ? 0x80008000u : 0u;
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const u32x4 p = {fA[e][0] ^ tm, fA[e][1] ^ tm, fA[e][2] ^ tm, fA[e][3] ^ tm};
                        Ap[e] = p;
                        An[e] = p ^ 0x80008000u;
                    }
                } else {
                    ts = neg_grp ? -1.f : 1.f;
                }
            }
            if constexpr (PLANES >= 2) {
                // plane-outer order: consecutive MFMAs never share an accumulator
#pragma unroll
                for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const bool neg = popc_const((uint32_t)rb & (uint32_t)(u >> 1)) & 1;
                        const u32x4 A = neg ? An[u & 1] : Ap[u & 1];
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[pl == 0 ? 0 : ACC - 1][rb][cb] =
                                mfma16<PLANES>(A, ring[slot][pl * 2 + cb], acc[pl == 0 ? 0 : ACC - 1][rb][cb]);
                    }
            } else {
                const f32x4 Bv[2] = {__builtin_bit_cast(f32x4, ring[slot][0]),
                                     __builtin_bit_cast(f32x4, ring[slot][1])};
#pragma unroll
                for (int t = 0; t < 4; ++t)
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) {
                        const bool neg = popc_const((uint32_t)rb & (uint32_t)(u >> 2)) & 1;
                        const float A = (neg ? -ts : ts) * fF[u & 3][t];
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[0][rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, Bv[cb][t], acc[0][rb][cb], 0, 0, 0);
                    }
            }
            if constexpr (PLANES == 1) {
                if constexpr (GSX % FLUSH_SLICES == 0) {
                    if (uu % FLUSH_SLICES == FLUSH_SLICES - 1) flush_into<RB>(tot, acc);
                } else {
                    if ((s0 + uu + 1) % FLUSH_SLICES == 0) flush_into<RB>(tot, acc);
                }
            }
            // Refill this slot with slice s+PF.  The fences keep the loads
            // here, PF slices ahead of their use, instead of letting the
            // scheduler sink them next to the MFMAs that consume them.
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (HERM) {
                // walk index s0+uu+PF lies in this step or the next, whose
                // slices are consecutive: a constant offset from sr or sn
                fetch(slot, uu + PF < GSX ? sr + (uint32_t)(uu + PF) : sn + (uint32_t)(uu + PF - GSX));
            } else {
                const uint32_t nxt = s0 + uu + PF;
                fetch(slot, nxt < nK ? nxt : nK - 1);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    };
    constexpr int GSL = (PLANES >= 2 && RB == 4 && DIR == FORWARD && !(PLANES == 2 && HERM)) ? 4 * GS : GS;
    // a half walk nests steps of GS slices (2^beta >= GS); the long step needs 2^beta >= GSL
    const bool long_ok = !half || (1u << beta) >= (uint32_t)GSL;
    if (active && nK % GSL == 0 && long_ok) {
        main_loop(std::integral_constant<int, GSL>{});
    } else if (active && nK % GS == 0) {
        main_loop(std::integral_constant<int, GS>{});
    } else if (active) {
        // Fewer K slices than one unrolled group (small matrices in a batch
        // whose tile shape was chosen for larger ones): one slice at a time,
        // signs evaluated at run time.  (A half walk never lands here.)
        for (uint32_t c = 0; c < nK; ++c) {
            const uint32_t s = slice_of(c);
            u32x4 B[P::NPL];
            const unsigned char* p = wsx + (size_t)s * P::SLICE_BYTES;
#pragma unroll
            for (int f = 0; f < P::NPL; ++f) B[f] = *(const u32x4*)(p + f * FRAG);
            const uint32_t qblk = (s * P::SK) >> 5;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const bool neg = __popc(((Pw >> 5) + rb) & qblk) & 1;
                if constexpr (PLANES >= 2) {
                    const uint32_t m = neg ? 0x80008000u : 0u;
                    const int e = s & 1;
                    const u32x4 A = u32x4{fA[e][0] ^ m, fA[e][1] ^ m, fA[e][2] ^ m, fA[e][3] ^ m};
#pragma unroll
                    for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
                        for (int cb = 0; cb < 2; ++cb)
                            acc[pl == 0 ? 0 : ACC - 1][rb][cb] =
                                mfma16<PLANES>(A, B[pl * 2 + cb], acc[pl == 0 ? 0 : ACC - 1][rb][cb]);
                } else {
                    const f32x4 B0 = __builtin_bit_cast(f32x4, B[0]), B1 = __builtin_bit_cast(f32x4, B[1]);
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float A = (neg ? -1.f : 1.f) * fF[s & 3][t];
                        acc[0][rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B0[t], acc[0][rb][0], 0, 0, 0);
                        acc[0][rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B1[t], acc[0][rb][1], 0, 0, 0);
                    }
                }
            }
            if constexpr (PLANES == 1) {
                if ((c + 1) % FLUSH_SLICES == 0) flush_into<RB>(tot, acc);
            }
        }
    }

    const double sc = half ? 2.0 * scale : scale;   // a half walk sums one member of each pair
    if constexpr (PLANES == 1) {
        flush_into<RB>(tot, acc);
        store_tile<PLANES, RB, DIR, HERM, herm_half_from(PLANES, RB, PF), (uint32_t)MT>(tot, dst, N, X0, Pw, sc, out128, lds);
    } else {
        store_tile<PLANES, RB, DIR, HERM, herm_half_from(PLANES, RB, PF), (uint32_t)MT>(acc, dst, N, X0, Pw, sc, out128, lds);
    }
}

// s_waitcnt (gfx9 encoding: vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8],
// vmcnt[15:14]).  Wait until at most NV vector-memory operations of this wave are outstanding
// and every LDS read it issued has returned (lgkmcnt 0), so that a following
// barrier also orders this wave's LDS reads before other waves' ring refills.
template <int NV>
__device__ inline void wait_vmcnt() {
    static_assert(NV >= 0 && NV < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((NV & 15) | (7 << 4) | (0 << 8) | ((NV >> 4) << 14));
}

// Variant of contract_tile for 4-wave workgroups that stages the packed
// operand once per workgroup: slices are handled in pairs, each pair's
// fragments are copied HBM/L2 -> LDS by direct loads (each wave copies a
// quarter, AHEAD pairs ahead of use, into a ring of AHEAD+1 pair slots), and
// all four waves read the B fragments from LDS.  Per pair: wait for this
// wave's own copies of the pair, one workgroup barrier (the pair is complete
// and the slot refilled next held a pair every wave has finished), refill,
// then the MFMAs.  lds must hold max(ring, epilogue staging) bytes.
template <int PLANES, int RB, int DIR, int AHEAD>
__device__ __attribute__((always_inline)) inline void contract_tile_lds(const unsigned char* __restrict__ wsm, unsigned char* __restrict__ dst,
                                         int N, uint32_t xb, uint32_t mb, double scale, int out128,
                                         unsigned char* lds) {
    using P = Pack<PLANES>;
    constexpr int WAVES = 4;
    constexpr int ACC = P::ACC;
    constexpr int MT = WAVES * RB * 32;
    constexpr int PAIR_FR = 2 * P::NPL;                    // fragments per slice pair
    constexpr int LPW = PAIR_FR / WAVES;                   // copies per wave per pair
    static_assert(PAIR_FR % WAVES == 0, "pair must split evenly over the waves");
    constexpr int PAIR_BYTES = PAIR_FR * FRAG;
    constexpr int NSL = AHEAD + 1;                         // ring slots
    constexpr int U = 32 * RB / P::SK;                     // slices per sign group
    constexpr int GP = U / 2;                              // pairs per sign group
    static_assert(U % 2 == 0, "sign group holds whole pairs");

    const uint32_t Dp = padded_dim(N);
    const uint32_t nS = Dp / P::SK, nP = nS / 2;
    const uint32_t X0 = xb * XT;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l32 = lane & 31, h = lane >> 5;
    const uint32_t Pw = mb * MT + wave * RB * 32;
    const unsigned char* slab = wsm + (size_t)xb * nS * P::SLICE_BYTES;   // pairs are contiguous

    uint32_t fA[2][4];
    float fF[4][4];
    if constexpr (PLANES >= 2) {
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                const uint32_t q0 = 16 * e + 8 * h + 2 * jj;
                const uint32_t s0 = ONE16<PLANES> | ((__popc(l32 & q0) & 1) ? 0x8000u : 0u);
                const uint32_t s1 = ONE16<PLANES> | ((__popc(l32 & (q0 + 1)) & 1) ? 0x8000u : 0u);
                fA[e][jj] = s0 | (s1 << 16);
            }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int t = 0; t < 4; ++t)
                fF[e][t] = (__popc(l32 & (8 * e + 4 * h + t)) & 1) ? -1.f : 1.f;
    }
    f32x16 acc[ACC][RB][2], tot[1][RB][2];   // tot: binary32 plane's flushed total
#pragma unroll
    for (int a = 0; a < ACC; ++a)
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[a][rb][cb][r] = tot[0][rb][cb][r] = 0.f;

    // copy this wave's quarter of pair p (clamped to the last pair) into its slot
    auto copy_pair = [&](uint32_t p, uint32_t slot) {
        const uint32_t ps = p < nP ? p : nP - 1;
        const unsigned char* g = slab + (size_t)ps * PAIR_BYTES + (wave * LPW) * FRAG + lane * 16;
        unsigned char* l = lds + slot * PAIR_BYTES + (wave * LPW) * FRAG;
#pragma unroll
        for (int j = 0; j < LPW; ++j)
            __builtin_amdgcn_global_load_lds(g + j * FRAG, (__attribute__((address_space(3))) void*)(l + j * FRAG),
                                             16, 0, 0);
    };
    // B fragments of one pair (two slices) as read from LDS, ping-ponged so the
    // next pair's reads go out half-way through the current pair's MFMAs.
    u32x4 Bb[2][2][P::NPL];
    auto read_pair = [&](uint32_t p, int buf) {
        const unsigned char* base = lds + (p % NSL) * PAIR_BYTES + lane * 16;
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int f = 0; f < P::NPL; ++f) Bb[buf][k][f] = *(const u32x4*)(base + (k * P::NPL + f) * FRAG);
    };
    u32x4 Ap[2], An[2];
    float ts = 1.f;
    auto slice_mfma = [&](int buf, int k, int u) {
        if constexpr (PLANES >= 2) {
#pragma unroll
            for (int pl = 0; pl < PLANES; ++pl)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const bool neg = popc_const((uint32_t)rb & (uint32_t)(u >> 1)) & 1;
                    const u32x4 A = neg ? An[u & 1] : Ap[u & 1];
#pragma unroll
                    for (int cb = 0; cb < 2; ++cb)
                        acc[pl == 0 ? 0 : ACC - 1][rb][cb] =
                            mfma16<PLANES>(A, Bb[buf][k][pl * 2 + cb], acc[pl == 0 ? 0 : ACC - 1][rb][cb]);
                }
        } else {
            const f32x4 B0 = __builtin_bit_cast(f32x4, Bb[buf][k][0]), B1 = __builtin_bit_cast(f32x4, Bb[buf][k][1]);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const bool neg = popc_const((uint32_t)rb & (uint32_t)(u >> 2)) & 1;
                    const float A = (neg ? -ts : ts) * fF[u & 3][t];
                    acc[0][rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B0[t], acc[0][rb][0], 0, 0, 0);
                    acc[0][rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(A, B1[t], acc[0][rb][1], 0, 0, 0);
                }
        }
    };

    // Prologue: copies of pairs 0..AHEAD in flight, pair 0 complete and read.
#pragma unroll
    for (int k = 0; k <= AHEAD; ++k) copy_pair(k, k);
    wait_vmcnt<LPW * AHEAD>();
    __builtin_amdgcn_s_barrier();
    read_pair(0, 0);

    static_assert(GP % 2 == 0 || GP == 1, "ping-pong over the pairs of a sign group");
    for (uint32_t p0 = 0; p0 < nP; p0 += GP) {
        const bool neg_grp = __popc((Pw >> 5) & ((2 * p0 * P::SK) >> 5)) & 1;
        if constexpr (PLANES >= 2) {
            const uint32_t tm = neg_grp ? 0x80008000u : 0u;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const u32x4 q = {fA[e][0] ^ tm, fA[e][1] ^ tm, fA[e][2] ^ tm, fA[e][3] ^ tm};
                Ap[e] = q;
                An[e] = q ^ 0x80008000u;
            }
        } else {
            ts = neg_grp ? -1.f : 1.f;
        }
#pragma unroll
        for (int j = 0; j < GP; ++j) {
            const uint32_t p = p0 + j;
            const int cur = (GP == 1) ? (int)(p & 1) : (j & 1);
            __builtin_amdgcn_sched_barrier(0);
            slice_mfma(cur, 0, 2 * j);
            __builtin_amdgcn_sched_barrier(0);
            // mid-pair: pair p+1 complete everywhere; refill the slot pair p
            // used (its fragments are in registers); read pair p+1.
            wait_vmcnt<LPW * (AHEAD - 1)>();
            __builtin_amdgcn_s_barrier();
            copy_pair(p + 1 + AHEAD, (p + 1 + AHEAD) % NSL);
            read_pair(p + 1, cur ^ 1);
            __builtin_amdgcn_sched_barrier(0);
            slice_mfma(cur, 1, 2 * j + 1);
            if constexpr (PLANES == 1) {
                if ((2 * (p + 1)) % FLUSH_SLICES == 0) flush_into<RB>(tot, acc);
            }
        }
    }
    wait_vmcnt<0>();                    // the ring's last (unused) copies land before the
    __builtin_amdgcn_s_barrier();       // epilogue reuses the LDS
    if constexpr (PLANES == 1) {
        flush_into<RB>(tot, acc);
        store_tile<PLANES, RB, DIR>(tot, dst, N, X0, Pw, scale, out128, lds);
    } else {
        store_tile<PLANES, RB, DIR>(acc, dst, N, X0, Pw, scale, out128, lds);
    }
}

}  // namespace mfma
}  // namespace pauli
