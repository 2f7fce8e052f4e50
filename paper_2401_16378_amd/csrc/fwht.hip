// All 4^N coefficients by fast Walsh-Hadamard transforms, O(N 4^N), in
// binary64 -- not the paper's O(8^N) evaluation but the same result: for
// every flip mask x the coefficients c(x, .) are the Sylvester-Hadamard
// transform of the gathered diagonal v_x[i] = G[i^x][i] followed by the
// phase (-i)^{popc(x&z)} and 2^-N (T. Jones 2024, section 2,
// Eq. (c_def_in_terms_of_fn) with the Pauli matrices of Eq. (3)).
//
// With i = 32 i_h + i_l and z = 32 z_h + z_l the sign (-1)^{popc(i&z)}
// factors into (-1)^{popc(i_l&z_l)} (-1)^{popc(i_h&z_h)}, so the transform
// splits into two HBM passes through a binary64 intermediate
//   U(x, z_l, i_h) = sum_{i_l} (-1)^{popc(i_l&z_l)} G[(32 i_h + i_l)^x][32 i_h + i_l]
//   c(x, 32 z_h + z_l) = 2^-N (-i)^{popc(x&z)} sum_{i_h} (-1)^{popc(i_h&z_h)} U(x, z_l, i_h)
// (U holds 4^N complex binary64 values, 16 bytes each, in the workspace,
// stored as U[x][i_h / 8][z_l][i_h % 8] so that both passes move long
// contiguous runs).
//
// Pass 1: a workgroup owns 32 flip masks x0..x0+31 and 8 consecutive i_h,
// whose eight tiles it requests together (four at a time for complex128).
// For each i_h the 32 x 32 block of G at rows (32 i_h ^ x0) .. +31, columns
// 32 i_h .. +31 holds exactly the 32 diagonals' entries for those i (entry
// (r, c) belongs to x_l = r ^ c, i_l = c), so it is loaded whole, widened to
// binary64 in LDS, and read back transposed: thread t takes x_l = t >> 3 and
// i_l = 4 (t & 7) + k, k < 4.  The 32-point butterflies run over k inside the
// thread and over lanes t ^ 1, t ^ 2, t ^ 4 (i_l bits 2..4).  The workgroup's
// results for one flip mask (32 z_l x 8 i_h) are one contiguous 4 KiB block
// of U.
//
// Pass 2: a workgroup owns 16 vectors U(x, z_l, .) -- 4 flip masks x_l =
// 4a..4a+3 and 4 phase values z_l = 4b..4b+3 of one 32-mask block -- with
// TPV (up to 64) threads per vector holding i_h = q + TPV k.  Butterflies run
// over k in the thread and over lanes q ^ 1, 2, ..., TPV / 2.  For each z_h the 16 results are
// the 16 consecutive coefficients n with fixed high bits (n's low four bits
// are (x^z)_0, z_0, (x^z)_1, z_1), so they are staged in LDS and stored as one
// contiguous 128-byte (complex64) or 256-byte (complex128) run.  For vectors
// of 512 (N >= 14) lane exchanges would dominate, so that pass runs 4 bits in
// the thread, one bit between lane pairs and, after a transpose through LDS,
// the last 4 bits in the thread again.
//
// Butterflies across lanes use DPP moves (partners 1 and 2 lanes apart, and 8
// within a row of 16) or ds_swizzle (4 and 16 apart), with the sum or the
// difference picked by one fma with a +-1 factor: the same rounding as an add
// or a subtract.
//
// The intermediate is binary64 (PAULI_ALGO_FWHT) or binary32
// (PAULI_ALGO_FWHT_F32: half the bytes; U is rounded once to binary32 after
// pass 1, and once more after each extra top pass at N = 15, 16, while every
// sum is still formed in binary64).
#include <type_traits>

#include "common.hpp"
#include "internal.hpp"

namespace pauli {
namespace {

constexpr int HB = 8;                   // i_h values per pass-1 workgroup


typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ inline double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// Value of lane ^ M (M < 32): DPP quad permutations for 1 and 2, a rotation
// by 8 within the row of 16 for 8, ds_swizzle (xor mode, 32-lane groups) for
// 4 and 16.
template <int M>
__device__ inline int lane_xor(int v) {
    static_assert(M == 1 || M == 2 || M == 4 || M == 8 || M == 16, "lane distance");
    if constexpr (M == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    else if constexpr (M == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    else if constexpr (M == 8) return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror 8
    else return __builtin_amdgcn_ds_swizzle(v, 0x1F | (M << 10));
}

template <int M>
__device__ inline double lane_xor_f64(double v) {
    return __hiloint2double(lane_xor<M>(__double2hiint(v)), lane_xor<M>(__double2loint(v)));
}

// Butterfly across lanes on the index bit owned by lane bit M: the lane whose
// M-bit is clear keeps a + b, its partner keeps a - b.
template <int M>
__device__ inline double2 lane_butterfly(double2 v, int lane) {
    const double sg = (lane & M) ? -1.0 : 1.0;
    const double px = lane_xor_f64<M>(v.x), py = lane_xor_f64<M>(v.y);
    return make_double2(__fma_rn(sg, v.x, px), __fma_rn(sg, v.y, py));
}

// The butterflies over lane bits 1 .. TPV / 2 of every value a thread holds.
template <int TPV, int EPT>
__device__ inline void lane_stages(double2 (&v)[EPT], int lane) {
    if constexpr (TPV > 1) {
        lane_stages<TPV / 2, EPT>(v, lane);
#pragma unroll
        for (int k = 0; k < EPT; ++k) v[k] = lane_butterfly<TPV / 2>(v[k], lane);
    }
}

// In-thread butterflies over all log2(EPT) bits of k.
template <int EPT>
__device__ inline void thread_stages(double2 (&v)[EPT]) {
#pragma unroll
    for (int s = 1; s < EPT; s <<= 1)
#pragma unroll
        for (int k = 0; k < EPT; ++k)
            if ((k & s) == 0) {
                const double2 p = v[k], r = v[k + s];
                v[k] = add2(p, r);
                v[k + s] = sub2(p, r);
            }
}

// The intermediate U (or W): binary64 or binary32 pairs, summed in binary64.
__device__ inline void put_u(double2* p, double2 v) { *p = v; }
__device__ inline void put_u(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ inline double2 get_u(const double2* p) { return *p; }
__device__ inline double2 get_u(const float2* p) {
    const float2 f = *p;
    return make_double2((double)f.x, (double)f.y);
}

template <bool IN128>
__device__ inline double2 load_g(const void* G, size_t idx) {
    if constexpr (IN128) {
        return ((const double2*)G)[idx];
    } else {
        const float2 g = ((const float2*)G)[idx];
        return make_double2((double)g.x, (double)g.y);
    }
}

template <bool IN128, typename UT>
__global__ __launch_bounds__(256) void fwht_pass1(const void* __restrict__ Gall, UT* __restrict__ Uall, int N) {
    using InT = typename std::conditional<IN128, double2, float2>::type;
    constexpr int PF = IN128 ? 4 : 8;    // tiles whose loads are issued together (32 or 64 KiB per workgroup)
    __shared__ double2 tile[32 * 33];    // [row][column], padded row
    const uint32_t D = 1u << N, M = D >> 5;
    const uint32_t x0 = blockIdx.y * 32u, h0 = blockIdx.x * HB;
    const size_t mat = (size_t)D * D;
    const InT* G = (const InT*)Gall + (size_t)blockIdx.z * mat;
    UT* U = Uall + (size_t)blockIdx.z * mat;
    const int t = threadIdx.x, lane = t & 63;
    const int lr = t >> 3, lc = (t & 7) * 4;       // load: row, first column of 4
    const int xl = t >> 3, il0 = (t & 7) * 4;      // transform: flip mask, first i_l of 4

    double2 acc[4][HB];
#pragma unroll
    for (int h1 = 0; h1 < HB; h1 += PF) {
        InT g[PF][4];
#pragma unroll
        for (int h = 0; h < PF; ++h) {
            const uint32_t ih = h0 + h1 + h;
            const uint32_t row = ((ih << 5) ^ x0) + lr, col = (ih << 5) + lc;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const InT e = G[(size_t)row * D + col + k];
                g[h][k].x = e.x;
                g[h][k].y = e.y;
            }
        }
#pragma unroll
        for (int h = 0; h < PF; ++h) {
            if (h1 + h > 0) __syncthreads();     // previous tile fully read
#pragma unroll
            for (int k = 0; k < 4; ++k) tile[lr * 33 + lc + k] = make_double2((double)g[h][k].x, (double)g[h][k].y);
            __syncthreads();
            double2 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int il = il0 + k;
                v[k] = tile[(il ^ xl) * 33 + il];
            }
            // i_l bits 0 and 1: inside the thread
            {
                const double2 a0 = add2(v[0], v[1]), a1 = sub2(v[0], v[1]);
                const double2 a2 = add2(v[2], v[3]), a3 = sub2(v[2], v[3]);
                v[0] = add2(a0, a2);
                v[2] = sub2(a0, a2);
                v[1] = add2(a1, a3);
                v[3] = sub2(a1, a3);
            }
            // i_l bits 2, 3, 4: lanes t ^ 1, t ^ 2, t ^ 4
            lane_stages<8, 4>(v, lane);
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k][h1 + h] = v[k];
        }
    }
    // U block (x, i_h / 8): [z_l][i_h % 8], 4 KiB contiguous per flip mask
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t zl = il0 + k;
        UT* dst = U + (((size_t)(x0 + xl) * (M / HB) + blockIdx.x) * 32u + zl) * HB;
#pragma unroll
        for (int h = 0; h < HB; ++h) put_u(dst + h, acc[k][h]);
    }
}

// TPV threads per vector (16 or 32), EPT elements per thread: the
// workgroup transforms ML = TPV EPT values of i_h per vector (all 2^(N-5)
// of them up to N = 14; above, each of the 2^(N-14) blocks of 512 whose top
// bits fwht_top has already transformed, selected by blockIdx.x >> 6); the
// workgroup has 16 TPV threads.
//
// ML < 512: thread q holds i_h = q + TPV k; butterflies over k in the thread,
// then over lanes q ^ 1, ..., TPV / 2.
// ML = 512 (TPV = 32, EPT = 16): thread q first holds i_h = (q >> 1) +
// 16 (q & 1) + 32 k: bits 5..8 (k) in the thread, bit 4 between lanes q and
// q ^ 1; an LDS transpose (real parts, then imaginary parts, rows padded by
// one double per 16) then gives it i_h = 16 (q & 1) + 32 (q >> 1) + j for
// bits 0..3 (j) in the thread.
constexpr uint32_t TR_PITCH = 512 + 32;   // doubles per vector row of the transpose

// The output stage holds one row of 16 coefficients per z_h (16 ESZ bytes).
// The threads writing one stage instruction hold rows 16 apart (transposing
// shape) or consecutive rows (the others), which would all fall on the same
// LDS banks; 16 bytes of padding after every PADR rows spread them.
template <bool TRANSPOSE, int ESZ>
constexpr uint32_t stage_pad_rows() { return TRANSPOSE ? 16u : (ESZ == 16 ? 1u : 2u); }

template <bool TRANSPOSE, int ESZ>
__device__ inline uint32_t stage_row(uint32_t zh) {
    return zh * 16u * ESZ + (zh / stage_pad_rows<TRANSPOSE, ESZ>()) * 16u;
}

template <bool TRANSPOSE, int ESZ>
constexpr size_t stage_bytes(uint32_t ML) {
    return (size_t)ML * 16u * ESZ + (size_t)(ML / stage_pad_rows<TRANSPOSE, ESZ>()) * 16u;
}

template <int TPV, int EPT, bool OUT128>
constexpr size_t pass2_lds_bytes() {
    constexpr bool T = TPV * EPT == 512;
    const size_t stage = stage_bytes<T, OUT128 ? 16 : 8>(TPV * EPT);
    const size_t tr = T ? 16u * TR_PITCH * 8u : 0u;
    return stage > tr ? stage : tr;
}

template <int TPV, int EPT, bool OUT128, typename UT>
__global__ __launch_bounds__(16 * TPV) void fwht_pass2(const UT* __restrict__ Uall, void* __restrict__ outall,
                                                       int N, double scale) {
    extern __shared__ __attribute__((aligned(16))) unsigned char stage[];   // [z_h][16] coefficients
    constexpr uint32_t ML = (uint32_t)TPV * EPT;
    constexpr bool TRANSPOSE = ML == 512;
    static_assert(!TRANSPOSE || (TPV == 32 && EPT == 16), "transposing shape");
    constexpr int ESZ = OUT128 ? 16 : 8;
    constexpr uint32_t NT = 16u * TPV;
    const uint32_t D = 1u << N, M = D >> 5;
    const size_t mat = (size_t)D * D;
    const uint32_t x0 = blockIdx.y * 32u;
    const uint32_t a = blockIdx.x & 7u, b = (blockIdx.x >> 3) & 7u;   // x_l quad, z_l quad
    const uint32_t h0 = (blockIdx.x >> 6) * ML;                       // first i_h (and z_h) of this block
    const UT* U = Uall + (size_t)blockIdx.z * mat;
    unsigned char* out = (unsigned char*)outall + (size_t)blockIdx.z * mat * ESZ;
    const int t = threadIdx.x, lane = t & 63;
    const int vec = t / TPV, q = t % TPV;
    const uint32_t xl = 4u * a + (uint32_t)(vec & 3), zl = 4u * b + (uint32_t)(vec >> 2);
    const uint32_t x = x0 + xl;
    // i_h (relative to h0) of value k in the thread: before (first) and after (second) the transform
    const uint32_t q0 = TRANSPOSE ? ((uint32_t)q >> 1) + 16u * ((uint32_t)q & 1u) : (uint32_t)q;
    const uint32_t jb = 16u * ((uint32_t)q & 1u) + 32u * ((uint32_t)q >> 1);

    double2 v[EPT];
    const UT* src = U + (size_t)x * 32u * M + zl * HB;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t ih = h0 + q0 + (uint32_t)TPV * k;
        v[k] = get_u(src + (size_t)(ih / HB) * 32u * HB + ih % HB);
    }
    thread_stages<EPT>(v);   // high i_h bits: over k inside the thread
    if constexpr (TRANSPOSE) {
        // bit 4: lane pairs
#pragma unroll
        for (int k = 0; k < EPT; ++k) v[k] = lane_butterfly<1>(v[k], lane);
        double* row = (double*)stage + (uint32_t)vec * TR_PITCH;
#pragma unroll
        for (int part = 0; part < 2; ++part) {
            if (part) __syncthreads();            // real parts read back before the imaginary ones land
#pragma unroll
            for (int k = 0; k < EPT; ++k) {
                const uint32_t ih = q0 + 32u * k;
                row[ih + (ih >> 4)] = part ? v[k].y : v[k].x;
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < EPT; ++j) {
                const uint32_t ih = jb + j;
                if (part) v[j].y = row[ih + (ih >> 4)];
                else v[j].x = row[ih + (ih >> 4)];
            }
        }
        thread_stages<EPT>(v);   // bits 0..3
        __syncthreads();          // transpose reads done before the stage reuses the LDS
    } else {
        // low i_h bits: lanes q ^ 1, 2, ..., TPV / 2 (a vector's threads are consecutive lanes of one wave)
        lane_stages<TPV, EPT>(v, lane);
    }

    // phase, scale, stage: slot = (x^z)_0 | z_0 << 1 | (x^z)_1 << 2 | z_1 << 3
    const uint32_t slot = ((xl ^ zl) & 1u) | ((zl & 1u) << 1) | (((xl ^ zl) & 2u) << 1) | ((zl & 2u) << 2);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t zh = TRANSPOSE ? jb + (uint32_t)k : (uint32_t)q + (uint32_t)TPV * k;   // row of the stage
        const uint32_t z = ((h0 + zh) << 5) + zl;
        double re = v[k].x * scale, im = v[k].y * scale;
        rotate_minus_i(re, im, (uint32_t)__popc(x & z));
        unsigned char* dstl = stage + stage_row<TRANSPOSE, ESZ>(zh) + slot * ESZ;
        if constexpr (OUT128) *(double2*)dstl = make_double2(re, im);
        else *(float2*)dstl = make_float2((float)re, (float)im);
    }
    __syncthreads();
    // ML runs of 16 coefficients (16 * ESZ bytes each), 16-byte stores
    constexpr uint32_t CH = (16u * ESZ) / 16u;    // 16-byte chunks per run
    const uint32_t xb4 = x0 + 4u * a, zb4 = 4u * b;
    for (uint32_t j = (uint32_t)t; j < ML * CH; j += NT) {
        const uint32_t zh = j / CH, part = j % CH;
        const uint32_t base = pauli_index(xb4, ((h0 + zh) << 5) + zb4);   // low four bits are zero
        *(u32x4_t*)(out + (size_t)base * ESZ + part * 16u) =
            *(const u32x4_t*)(stage + stage_row<TRANSPOSE, ESZ>(zh) + part * 16u);
    }
}

// ---- adjoint: G[i^x][i] = scale sum_z i^{popc(x&z)} (-1)^{popc(i&z)} c(x, z) ----
// Pass A mirrors pass 2: the 16 coefficient runs of a workgroup's vectors are
// read into LDS, phased by i^{popc(x&z)}, transformed over z_h (H is
// symmetric, so the same butterflies map z_h to i_h) and stored as
// W(x, z_l, i_h) in U's blocked layout.
template <int TPV, int EPT, bool IN128, typename UT>
__global__ __launch_bounds__(16 * TPV) void fwht_adj_a(const void* __restrict__ inall, UT* __restrict__ Wall, int N) {
    extern __shared__ __attribute__((aligned(16))) unsigned char stage[];   // [z_h][16] coefficients
    constexpr uint32_t ML = (uint32_t)TPV * EPT;
    constexpr int ESZ = IN128 ? 16 : 8;
    constexpr uint32_t NT = 16u * TPV;
    const uint32_t D = 1u << N, M = D >> 5;
    const size_t mat = (size_t)D * D;
    const uint32_t x0 = blockIdx.y * 32u;
    const uint32_t a = blockIdx.x & 7u, b = (blockIdx.x >> 3) & 7u;
    const uint32_t h0 = (blockIdx.x >> 6) * ML;
    const unsigned char* in = (const unsigned char*)inall + (size_t)blockIdx.z * mat * ESZ;
    UT* W = Wall + (size_t)blockIdx.z * mat;
    const int t = threadIdx.x, lane = t & 63;
    const int vec = t / TPV, q = t % TPV;
    const uint32_t xl = 4u * a + (uint32_t)(vec & 3), zl = 4u * b + (uint32_t)(vec >> 2);
    const uint32_t x = x0 + xl;

    constexpr uint32_t CH = (16u * ESZ) / 16u;
    const uint32_t xb4 = x0 + 4u * a, zb4 = 4u * b;
    for (uint32_t j = (uint32_t)t; j < ML * CH; j += NT) {
        const uint32_t zh = j / CH, part = j % CH;
        const uint32_t base = pauli_index(xb4, ((h0 + zh) << 5) + zb4);
        *(u32x4_t*)(stage + stage_row<false, ESZ>(zh) + part * 16u) =
            *(const u32x4_t*)(in + (size_t)base * ESZ + part * 16u);
    }
    __syncthreads();
    const uint32_t slot = ((xl ^ zl) & 1u) | ((zl & 1u) << 1) | (((xl ^ zl) & 2u) << 1) | ((zl & 2u) << 2);
    double2 v[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t zh = (uint32_t)q + (uint32_t)TPV * k;
        const uint32_t z = ((h0 + zh) << 5) + zl;
        const unsigned char* src = stage + stage_row<false, ESZ>(zh) + slot * ESZ;
        double re, im;
        if constexpr (IN128) {
            const double2 c = *(const double2*)src;
            re = c.x;
            im = c.y;
        } else {
            const float2 c = *(const float2*)src;
            re = (double)c.x;
            im = (double)c.y;
        }
        rotate_minus_i(re, im, 3u * (uint32_t)__popc(x & z));   // i^{popc(x&z)}
        v[k] = make_double2(re, im);
    }
    thread_stages<EPT>(v);
    lane_stages<TPV, EPT>(v, lane);
    UT* dst = W + (size_t)x * 32u * M + zl * HB;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t ih = h0 + (uint32_t)q + (uint32_t)TPV * k;
        put_u(dst + (size_t)(ih / HB) * 32u * HB + ih % HB, v[k]);
    }
}

// Pass B mirrors pass 1: for 32 flip masks and 8 consecutive i_h, the
// 32-point transforms over z_l give the diagonal entries y(x, 32 i_h + i_l),
// which an LDS tile turns back into the 32 x 32 block of G at rows
// (32 i_h ^ x0) .. +31, columns 32 i_h .. +31 (entry (r, c) holds x_l = r ^ c,
// i_l = c), written row by row.
template <bool OUT128, typename UT>
__global__ __launch_bounds__(256) void fwht_adj_b(const UT* __restrict__ Wall, void* __restrict__ Gall, int N,
                                                  double scale) {
    __shared__ double2 tile[32 * 33];
    const uint32_t D = 1u << N, M = D >> 5;
    const uint32_t x0 = blockIdx.y * 32u, h0 = blockIdx.x * HB;
    const size_t mat = (size_t)D * D;
    const UT* W = Wall + (size_t)blockIdx.z * mat;
    unsigned char* G = (unsigned char*)Gall + (size_t)blockIdx.z * mat * (OUT128 ? 16 : 8);
    const int t = threadIdx.x, lane = t & 63;
    const int xl = t >> 3, zl0 = (t & 7) * 4;      // transform: flip mask, first z_l of 4
    const int lr = t >> 3, lc = (t & 7) * 4;       // store: row, first column of 4

    double2 w[4][HB];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const UT* src = W + (((size_t)(x0 + xl) * (M / HB) + blockIdx.x) * 32u + zl0 + k) * HB;
#pragma unroll
        for (int h = 0; h < HB; ++h) w[k][h] = get_u(src + h);
    }
#pragma unroll
    for (int h = 0; h < HB; ++h) {
        double2 v[4] = {w[0][h], w[1][h], w[2][h], w[3][h]};
        {
            const double2 a0 = add2(v[0], v[1]), a1 = sub2(v[0], v[1]);
            const double2 a2 = add2(v[2], v[3]), a3 = sub2(v[2], v[3]);
            v[0] = add2(a0, a2);
            v[2] = sub2(a0, a2);
            v[1] = add2(a1, a3);
            v[3] = sub2(a1, a3);
        }
        lane_stages<8, 4>(v, lane);
        if (h > 0) __syncthreads();              // previous tile fully written out
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int il = zl0 + k;
            tile[(il ^ xl) * 33 + il] = make_double2(v[k].x * scale, v[k].y * scale);
        }
        __syncthreads();
        const uint32_t ih = h0 + h;
        const uint32_t row = ((ih << 5) ^ x0) + lr, col = (ih << 5) + lc;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double2 g = tile[lr * 33 + lc + k];
            if constexpr (OUT128) ((double2*)G)[(size_t)row * D + col + k] = g;
            else ((float2*)G)[(size_t)row * D + col + k] = make_float2((float)g.x, (float)g.y);
        }
    }
}

template <int TPV, int EPT, typename UT>
hipError_t launch_adj_a(const void* in, bool in128, UT* W, int N, int batch, uint32_t nxb, hipStream_t s) {
    const uint32_t ntop = ((1u << N) >> 5) / (uint32_t)(TPV * EPT);
    const dim3 grid(64u * ntop, nxb, (uint32_t)batch);
    const size_t lds = in128 ? stage_bytes<false, 16>(TPV * EPT) : stage_bytes<false, 8>(TPV * EPT);
    hipError_t e;
    if (in128) {
        e = hipFuncSetAttribute((const void*)fwht_adj_a<TPV, EPT, true, UT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_adj_a<TPV, EPT, true, UT>), grid, dim3(16 * TPV), lds, s, in, W, N);
    } else {
        e = hipFuncSetAttribute((const void*)fwht_adj_a<TPV, EPT, false, UT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_adj_a<TPV, EPT, false, UT>), grid, dim3(16 * TPV), lds, s, in, W, N);
    }
    return hipGetLastError();
}

template <int TPV, int EPT, typename UT>
hipError_t launch_pass2(const UT* U, void* out, bool out128, int N, int batch, double scale, uint32_t nxb,
                        hipStream_t s) {
    const uint32_t ntop = ((1u << N) >> 5) / (uint32_t)(TPV * EPT);
    const dim3 grid(64u * ntop, nxb, (uint32_t)batch);   // the 64 quads of a mask block back to back
    hipError_t e;
    if (out128) {
        constexpr size_t lds = pass2_lds_bytes<TPV, EPT, true>();
        e = hipFuncSetAttribute((const void*)fwht_pass2<TPV, EPT, true, UT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_pass2<TPV, EPT, true, UT>), grid, dim3(16 * TPV), lds, s, U, out, N, scale);
    } else {
        constexpr size_t lds = pass2_lds_bytes<TPV, EPT, false>();
        e = hipFuncSetAttribute((const void*)fwht_pass2<TPV, EPT, false, UT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_pass2<TPV, EPT, false, UT>), grid, dim3(16 * TPV), lds, s, U, out, N, scale);
    }
    return hipGetLastError();
}

// ---- orders 15 and 16: the top T = N - 14 bits of i_h ----
// In U's blocked layout the D values of one flip mask are contiguous and
// their i_h top bits select D / 2^T-element sub-blocks, so the 2^T partners
// of an element lie D / 2^T apart; each thread does one 2^T-point
// butterfly in place (a pure streaming pass).  Pass 2 (or adjoint pass A)
// then handles the remaining 9 bits of each sub-block.
template <int T, typename UT>
__global__ __launch_bounds__(256) void fwht_top(UT* __restrict__ Uall, int N) {
    const uint32_t D = 1u << N;
    const size_t mat = (size_t)D * D;
    UT* U = Uall + (size_t)blockIdx.y * mat;
    const uint32_t lgS = (uint32_t)N - T;                  // sub-block length 2^lgS
    const size_t S = (size_t)1 << lgS, total = (size_t)D << lgS;
    for (size_t f = (size_t)blockIdx.x * 256u + threadIdx.x; f < total; f += (size_t)gridDim.x * 256u) {
        UT* p = U + ((f >> lgS) << N) + (f & (S - 1));
        double2 v[1 << T];
#pragma unroll
        for (int k = 0; k < (1 << T); ++k) v[k] = get_u(p + ((size_t)k << lgS));
        thread_stages<(1 << T)>(v);
#pragma unroll
        for (int k = 0; k < (1 << T); ++k) put_u(p + ((size_t)k << lgS), v[k]);
    }
}

template <typename UT>
hipError_t launch_top(UT* U, int N, int batch, hipStream_t s) {
    const dim3 grid(8192u, (uint32_t)batch);
    if (N == 15) hipLaunchKernelGGL((fwht_top<1, UT>), grid, dim3(256), 0, s, U, N);
    else if (N == 16) hipLaunchKernelGGL((fwht_top<2, UT>), grid, dim3(256), 0, s, U, N);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---- orders N <= 8: one kernel, everything in LDS ----
// A workgroup owns W = min(32, D) flip masks x0 .. x0 + W - 1 and every
// column: it gathers the D / W blocks of W x W entries (the same bijection:
// entry (r, c) of the block at rows (i0 ^ x0) .., columns i0 .. belongs to
// x_l = r ^ c, i = i0 + c) into v[x_l][i] in binary64 (forward), runs the
// log2(D) butterfly stages over i in LDS, then writes each W x W (x_l, z_l)
// block -- a contiguous run of W^2 coefficients -- phased and scaled.  The
// adjoint reads those runs, phases by i^{popc(x&z)}, transforms over z and
// scatters through the same blocks.
template <bool IN128, bool OUT128, int DIR>
__global__ __launch_bounds__(256) void fwht_small(const void* __restrict__ inall, void* __restrict__ outall, int N,
                                                  double scale) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
    double2* v = (double2*)lds_raw;               // [W][D]
    const uint32_t D = 1u << N, W = D < 32u ? D : 32u;
    const uint32_t lw = D < 32u ? (uint32_t)N : 5u;
    const uint32_t x0 = blockIdx.x * W;
    const size_t mat = (size_t)D * D;
    const int t = threadIdx.x;
    const uint32_t total = W * D;
    const unsigned char* in = (const unsigned char*)inall + (size_t)blockIdx.y * mat * (IN128 ? 16 : 8);
    unsigned char* out = (unsigned char*)outall + (size_t)blockIdx.y * mat * (OUT128 ? 16 : 8);
    auto load = [&](size_t idx) {
        if constexpr (IN128) return ((const double2*)in)[idx];
        const float2 g = ((const float2*)in)[idx];
        return make_double2((double)g.x, (double)g.y);
    };
    auto store = [&](size_t idx, double re, double im) {
        if constexpr (OUT128) ((double2*)out)[idx] = make_double2(re * scale, im * scale);
        else ((float2*)out)[idx] = make_float2((float)(re * scale), (float)(im * scale));
    };
    // run element o of block (x0, z_h): x_l and z_l from n's interleaved bits
    auto run_xz = [&](uint32_t o, uint32_t& xl, uint32_t& zl) {
        zl = compact_even(o >> 1);
        xl = compact_even(o) ^ zl;
    };
    if constexpr (DIR == FORWARD) {
        for (uint32_t e = t; e < total; e += 256) {
            const uint32_t c = e & (W - 1u), r = (e >> lw) & (W - 1u), b = e >> (2 * lw);
            const uint32_t i0 = b << lw;
            v[(r ^ c) * D + i0 + c] = load((size_t)((i0 ^ x0) + r) * D + i0 + c);
        }
    } else {
        for (uint32_t e = t; e < total; e += 256) {
            const uint32_t zh = e >> (2 * lw), o = e & (W * W - 1u);
            uint32_t xl, zl;
            run_xz(o, xl, zl);
            const uint32_t z = (zh << lw) + zl;
            double2 c = load((size_t)pauli_index(x0, zh << lw) + o);
            rotate_minus_i(c.x, c.y, 3u * (uint32_t)__popc((x0 + xl) & z));
            v[xl * D + z] = c;
        }
    }
    __syncthreads();
    for (uint32_t m = 1; m < D; m <<= 1) {        // butterflies over the column (or z) index
        for (uint32_t e = t; e < total / 2; e += 256) {
            const uint32_t row = e / (D / 2), k = e % (D / 2);
            const uint32_t lo = ((k & ~(m - 1u)) << 1) | (k & (m - 1u));
            double2* pa = v + row * D + lo;
            const double2 a = pa[0], b = pa[m];
            pa[0] = add2(a, b);
            pa[m] = sub2(a, b);
        }
        __syncthreads();
    }
    if constexpr (DIR == FORWARD) {
        for (uint32_t e = t; e < total; e += 256) {
            const uint32_t zh = e >> (2 * lw), o = e & (W * W - 1u);
            uint32_t xl, zl;
            run_xz(o, xl, zl);
            const uint32_t z = (zh << lw) + zl;
            double2 c = v[xl * D + z];
            rotate_minus_i(c.x, c.y, (uint32_t)__popc((x0 + xl) & z));
            store((size_t)pauli_index(x0, zh << lw) + o, c.x, c.y);
        }
    } else {
        for (uint32_t e = t; e < total; e += 256) {
            const uint32_t c = e & (W - 1u), r = (e >> lw) & (W - 1u), b = e >> (2 * lw);
            const uint32_t i0 = b << lw;
            const double2 y = v[(r ^ c) * D + i0 + c];
            store((size_t)((i0 ^ x0) + r) * D + i0 + c, y.x, y.y);
        }
    }
}

template <bool IN128, bool OUT128>
hipError_t launch_small(Dir dir, const void* in, void* out, int N, int batch, double scale, hipStream_t s) {
    const uint32_t D = 1u << N, W = D < 32u ? D : 32u;
    const size_t lds = (size_t)W * D * 16u;
    const dim3 grid(D / W, (uint32_t)batch);
    hipError_t e;
    if (dir == FORWARD) {
        e = hipFuncSetAttribute((const void*)fwht_small<IN128, OUT128, FORWARD>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_small<IN128, OUT128, FORWARD>), grid, dim3(256), lds, s, in, out, N, scale);
    } else {
        e = hipFuncSetAttribute((const void*)fwht_small<IN128, OUT128, ADJOINT>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((fwht_small<IN128, OUT128, ADJOINT>), grid, dim3(256), lds, s, in, out, N, scale);
    }
    return hipGetLastError();
}

// The two-pass path with intermediate U of type UT (double2 or float2).
template <typename UT>
hipError_t launch_two_pass(Dir dir, const void* in, bool in_c128, void* out, bool out_c128, int N, int batch,
                           double scale, UT* U, hipStream_t s) {
    const uint32_t D = 1u << N, M = D >> 5, nxb = D / 32u;
    const dim3 gt(M / HB, nxb, (uint32_t)batch);   // consecutive i_h groups back to back
    hipError_t e = hipSuccess;
    if (dir == FORWARD) {
        if (in_c128) hipLaunchKernelGGL((fwht_pass1<true, UT>), gt, dim3(256), 0, s, in, U, N);
        else hipLaunchKernelGGL((fwht_pass1<false, UT>), gt, dim3(256), 0, s, in, U, N);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        switch (N) {   // (threads per vector, elements per thread)
            case 9: return launch_pass2<16, 1>(U, out, out_c128, N, batch, scale, nxb, s);
            case 10: return launch_pass2<32, 1>(U, out, out_c128, N, batch, scale, nxb, s);
            case 11: return launch_pass2<32, 2>(U, out, out_c128, N, batch, scale, nxb, s);
            case 12: return launch_pass2<32, 4>(U, out, out_c128, N, batch, scale, nxb, s);
            case 13: return launch_pass2<32, 8>(U, out, out_c128, N, batch, scale, nxb, s);
            case 14: return launch_pass2<32, 16>(U, out, out_c128, N, batch, scale, nxb, s);
            case 15:
            case 16:
                if ((e = launch_top(U, N, batch, s)) != hipSuccess) return e;
                return launch_pass2<32, 16>(U, out, out_c128, N, batch, scale, nxb, s);
            default: return hipErrorInvalidValue;
        }
    }
    switch (N) {
        case 9: e = launch_adj_a<16, 1>(in, in_c128, U, N, batch, nxb, s); break;
        case 10: e = launch_adj_a<32, 1>(in, in_c128, U, N, batch, nxb, s); break;
        case 11: e = launch_adj_a<32, 2>(in, in_c128, U, N, batch, nxb, s); break;
        case 12: e = launch_adj_a<32, 4>(in, in_c128, U, N, batch, nxb, s); break;
        case 13: e = launch_adj_a<32, 8>(in, in_c128, U, N, batch, nxb, s); break;
        case 14: e = launch_adj_a<32, 16>(in, in_c128, U, N, batch, nxb, s); break;
        case 15:
        case 16:
            e = launch_adj_a<32, 16>(in, in_c128, U, N, batch, nxb, s);
            if (e == hipSuccess) e = launch_top(U, N, batch, s);
            break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (out_c128) hipLaunchKernelGGL((fwht_adj_b<true, UT>), gt, dim3(256), 0, s, U, out, N, scale);
    else hipLaunchKernelGGL((fwht_adj_b<false, UT>), gt, dim3(256), 0, s, U, out, N, scale);
    return hipGetLastError();
}

}  // namespace

bool fwht_supported(int N) { return N >= FWHT_N_MIN && N <= FWHT_N_MAX; }

size_t fwht_workspace_bytes(int N, int batch, bool narrow) {
    return N <= FWHT_SMALL_N_MAX ? 0 : ((size_t)1 << (2 * N)) * (narrow ? 8u : 16u) * (size_t)batch;
}

hipError_t launch_fwht(Dir dir, const void* in, bool in_c128, void* out, bool out_c128, int N, int batch,
                       double scale, bool narrow, void* ws, hipStream_t s) {
    if (!fwht_supported(N)) return hipErrorInvalidValue;
    if (N <= FWHT_SMALL_N_MAX) {
        if (in_c128) return out_c128 ? launch_small<true, true>(dir, in, out, N, batch, scale, s)
                                     : launch_small<true, false>(dir, in, out, N, batch, scale, s);
        return out_c128 ? launch_small<false, true>(dir, in, out, N, batch, scale, s)
                        : launch_small<false, false>(dir, in, out, N, batch, scale, s);
    }
    if (narrow) return launch_two_pass(dir, in, in_c128, out, out_c128, N, batch, scale, (float2*)ws, s);
    return launch_two_pass(dir, in, in_c128, out, out_c128, N, batch, scale, (double2*)ws, s);
}

}  // namespace pauli
